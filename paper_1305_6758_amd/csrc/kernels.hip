// kernels.hip -- HIP kernels (gfx950) of the multipath Metropolis engine for the classical
// O(3) Heisenberg model (arXiv:1305.6758, Sec. 2).
//
// One simulation path is a periodic L^3 lattice of unit spins swept with single-spin
// Metropolis moves; paths are independent of each other (Sec. 2), so a group of G lanes of
// one workgroup owns one path for all of its sweeps. Within a path the sweep
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
#include "philox.hpp"

#include <algorithm>
#include <string.h>
#include <type_traits>
#include <utility>

namespace mmc {
namespace {

// ------------------------------------------------------------------ precision policies
template <typename T> struct Arith;

// FP32: uniforms with 23 random bits, u = ((w >> 8) | 1) 2^-24, exact and never 0 or 1: the
// bit pattern 0x3F800000 | (w >> 9) (one alignbit) is 1 + (w >> 9) 2^-23, and subtracting
// 1 - 2^-24 from it is exact. Transcendental unit for sqrt, sin and cos (argument in
// revolutions, so phi / (2 pi) = u1 goes in directly) and exp2.
template <> struct Arith<float> {
    static __device__ __forceinline__ float uni(uint32_t w)
    {
        return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9)) - 0x1.fffffep-1f;
    }
    static __device__ __forceinline__ void sphere(uint32_t w0, uint32_t w1, float &x, float &y, float &z)
    {
        const float zz = fmaf(2.0f, uni(w0), -1.0f);  // 2 u0 - 1, exact
        const float r = __builtin_amdgcn_sqrtf(fmaf(-zz, zz, 1.0f));
        const float rev = uni(w1);
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

// ------------------------------------------------------------------ wave reductions
template <int CTRL>
__device__ __forceinline__ float dpp_plus(float v)
{
    const int s = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false);
    return v + __int_as_float(s);
}

// Sum over the 16 lanes of each DPP row, left in every lane of the row.
__device__ __forceinline__ float row_sum(float v)
{
    v = dpp_plus<0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_plus<0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_plus<0x141>(v);  // row_half_mirror
    v = dpp_plus<0x140>(v);  // row_mirror
    return v;
}

__device__ __forceinline__ double row_sum(double v)
{
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum over the 64 lanes of the wave (wave-uniform result).
__device__ __forceinline__ float wave_sum(float v)
{
    v = row_sum(v);
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

enum Map { COLZ = 0, FLAT = 1 };

// Where a path's spins live while it sweeps: all in device memory, all in LDS, colour 0 in
// LDS and colour 1 in device memory (sides whose lattice is too large for LDS but half of it
// is not: 22 <= L <= 30 in FP32), or only colour 0's x and y components in LDS (a third of
// the lattice: L = 32 and 34 in FP32).
enum Place { PL_MEM = 0, PL_LDS = 1, PL_SPLIT = 2, PL_SPLIT_XY = 3, PL_RING = 4, PL_HRING = 5, PL_RING2 = 6 };

// Everything a path group needs during its sweeps; path, key and counter word are
// wave-uniform (each wave belongs to one path group).
template <typename T>
struct GroupCtx {
    int L;                            // side (runtime copy; kernels with a compile-time L use that)
    uint32_t path, key0, key1, ctr3;  // ctr3 = instance << 8 (tag added per use)
    bool active;                      // path < n_paths
    int lane;                         // 0 .. G-1
    T *sp;                            // colour-0 spins of this path while sweeping (LDS or device memory)
    T *sp1;                           // colour-1 spins (sp + 3 L^3 / 2, or device memory when only
                                      // colour 0 is in LDS)
    T *sp0z;                          // colour-0 z components in device memory (PL_SPLIT_XY)
    double *shacc;                    // 16 doubles in LDS: the path's PathAcc while sweeping
    T *red;                           // LDS [16-lane rows of the group][4] measurement partials
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

__device__ __forceinline__ Site flat_site(int L, int h, int c)
{
    const int HL = L >> 1, PLANE = HL * L;
    const int col = h % PLANE;
    return make_site(L, col % HL, col / HL, h / PLANE, c);
}

// Coefficients of the acceptance test.
template <typename T>
struct Coef {
    T beta, J;  // FP64 path
    float q;    // FP32 path: beta J log2(e)
};

// Element i of a spin array. For arrays in device memory (DEV) the index becomes an unsigned
// 32-bit byte offset from the (wave-uniform) base, which the backend turns into a scalar base
// plus a 32-bit vector offset instead of a 64-bit address per lane and component; LDS arrays
// keep plain indexing, whose constant parts fold into the instructions' offset fields. The
// base is one colour-component array and i < L^3 / 2 <= 2^29 (instances are limited to
// L^3 <= 2^30), so even an FP64 byte offset stays below 2^32.
template <bool DEV, typename T>
__device__ __forceinline__ T &spin_at(T *base, int i)
{
    using Byte = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    if constexpr (DEV) return *reinterpret_cast<T *>(reinterpret_cast<Byte *>(base) + (uint32_t)i * (uint32_t)sizeof(T));
    else return base[i];
}

// Spins of the two colours as per-component arrays: own = the colour being updated, oth =
// the other one (its components are the neighbours). DEV: a bit per component (x, y, z) set
// when that component lives in device memory (addressing only; the arithmetic is the same).
template <typename T>
struct ColourView {
    T *own[3];
    const T *oth[3];
};

// One Metropolis attempt at site s of sweep k, with the operand reads given as functors
// (own(c): component c of the site's spin; nbr(c, n): component c of neighbour n, order -x,
// +x, -y, +y, -z, +z). Adds the resulting spin (and for the odd colour S . h) to the
// measurement partials and the accepted count of the wave to nacc. store(acc, new spin, old
// spin) writes the outcome.
template <typename T, bool ANG, typename Own, typename Nbr, typename Store>
__device__ __forceinline__ void update_site_f(const GroupCtx<T> &g, bool odd, const Site &s, uint32_t k,
                                              const Coef<T> &cf, T &pe, T &pmx, T &pmy, T &pmz,
                                              unsigned long long &nacc, Own &&own, Nbr &&nbr, Store &&store)
{
    const Words w = philox4x32_10((uint32_t)s.id, k, g.path, TAG_MET | g.ctr3, g.key0, g.key1);
    const T sx = own(0), sy = own(1), sz = own(2);
    T hx, hy, hz;
    if constexpr (std::is_same<T, double>::value) {
        // h = ((((S_-x + S_+x) + S_-y) + S_+y) + S_-z) + S_+z, the reference order.
        hx = nbr(0, 0);
        hy = nbr(1, 0);
        hz = nbr(2, 0);
#pragma unroll
        for (int n = 1; n < 6; ++n) {
            hx = hx + nbr(0, n);
            hy = hy + nbr(1, n);
            hz = hz + nbr(2, n);
        }
    } else {
        // FP32: pairwise tree (any order is a valid FP32 rounding of the same sum).
        T ax[6], ay[6], az[6];
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            ax[n] = nbr(0, n);
            ay[n] = nbr(1, n);
            az[n] = nbr(2, n);
        }
        hx = ((ax[0] + ax[1]) + (ax[2] + ax[3])) + (ax[4] + ax[5]);
        hy = ((ay[0] + ay[1]) + (ay[2] + ay[3])) + (ay[4] + ay[5]);
        hz = ((az[0] + az[1]) + (az[2] + az[3])) + (az[4] + az[5]);
    }
    T nx, ny, nz;
    if constexpr (ANG) Arith<T>::angles(w.w0, w.w1, nx, ny, nz);  // both angles uniform
    else Arith<T>::sphere(w.w0, w.w1, nx, ny, nz);
    const T dx = nx - sx, dy = ny - sy, dz = nz - sz;
    bool acc;
    if constexpr (std::is_same<T, double>::value) {
        // dE = -J ((dx hx + dy hy) + dz hz); accept iff u < exp(-beta dE).
        const double dE = -cf.J * ((dx * hx + dy * hy) + dz * hz);
        acc = Arith<double>::uni(w.w2) < exp(-cf.beta * dE);
    } else {
        // -beta dE = beta J (S' - S) . h; accept iff u < 2^(beta J log2(e) (S' - S) . h).
        const float dot = fmaf(dz, hz, fmaf(dy, hy, dx * hx));
        acc = Arith<float>::uni(w.w2) < __builtin_amdgcn_exp2f(cf.q * dot);
    }
    // (counted before the store: the ballot then reads the compare's mask as it is, instead of
    // a copy rebuilt after the store's branch)
    nacc += (unsigned long long)__popcll(__ballot(acc));
    store(acc, nx, ny, nz, sx, sy, sz);
    const T fx = acc ? nx : sx, fy = acc ? ny : sy, fz = acc ? nz : sz;
    pmx += fx;
    pmy += fy;
    pmz += fz;
    if (odd) {
        if constexpr (std::is_same<T, double>::value) pe = pe + ((fx * hx + fy * hy) + fz * hz);
        else pe = fmaf(fz, hz, fmaf(fy, hy, fmaf(fx, hx, pe)));
    }
}

// The same with the operands read from a colour view: OWN_DEV / OTH_DEV are bit masks of the
// own / other colour's components in device memory (update_site_v's store writes the new spin
// into the own arrays when accepted).
template <typename T, bool ANG, int OWN_DEV, int OTH_DEV, typename Store>
__device__ __forceinline__ void update_site_s(const GroupCtx<T> &g, const ColourView<T> &cv, bool odd, const Site &s,
                                              uint32_t k, const Coef<T> &cf, T &pe, T &pmx, T &pmy, T &pmz,
                                              unsigned long long &nacc, Store &&store)
{
    T *const ox = cv.own[0], *const oy = cv.own[1], *const oz = cv.own[2];
    const T *const tx = cv.oth[0], *const ty = cv.oth[1], *const tz = cv.oth[2];
    constexpr bool OX = OWN_DEV & 1, OY = OWN_DEV & 2, OZ = OWN_DEV & 4;
    constexpr bool TX = OTH_DEV & 1, TY = OTH_DEV & 2, TZ = OTH_DEV & 4;
    update_site_f<T, ANG>(
        g, odd, s, k, cf, pe, pmx, pmy, pmz, nacc,
        [&](int c) { return c == 0 ? spin_at<OX>(ox, s.h) : c == 1 ? spin_at<OY>(oy, s.h) : spin_at<OZ>(oz, s.h); },
        [&](int c, int n) {
            return c == 0 ? spin_at<TX>(tx, s.nb[n]) : c == 1 ? spin_at<TY>(ty, s.nb[n]) : spin_at<TZ>(tz, s.nb[n]);
        },
        store);
}

template <typename T, bool ANG = false, int OWN_DEV = 0, int OTH_DEV = 0>
__device__ __forceinline__ void update_site_v(const GroupCtx<T> &g, const ColourView<T> &cv, bool odd, const Site &s,
                                              uint32_t k, const Coef<T> &cf, T &pe, T &pmx, T &pmy, T &pmz,
                                              unsigned long long &nacc)
{
    T *const ox = cv.own[0], *const oy = cv.own[1], *const oz = cv.own[2];
    constexpr bool OX = OWN_DEV & 1, OY = OWN_DEV & 2, OZ = OWN_DEV & 4;
    const int h = s.h;
    update_site_s<T, ANG, OWN_DEV, OTH_DEV>(g, cv, odd, s, k, cf, pe, pmx, pmy, pmz, nacc,
                                            [&](bool acc, T nx, T ny, T nz, T, T, T) {
                                                if (acc) {
                                                    spin_at<OX>(ox, h) = nx;
                                                    spin_at<OY>(oy, h) = ny;
                                                    spin_at<OZ>(oz, h) = nz;
                                                }
                                            });
}

// The same with each colour's components HALF apart (one array per colour, all in LDS or all
// in device memory).
template <typename T, bool ANG = false, bool OWN_DEV = false, bool OTH_DEV = false>
__device__ __forceinline__ void update_site(const GroupCtx<T> &g, T *own, const T *oth, int HALF, bool odd,
                                            const Site &s, uint32_t k, const Coef<T> &cf, T &pe, T &pmx, T &pmy,
                                            T &pmz, unsigned long long &nacc)
{
    const ColourView<T> cv{{own, own + HALF, own + 2 * HALF}, {oth, oth + HALF, oth + 2 * HALF}};
    update_site_v<T, ANG, OWN_DEV ? 7 : 0, OTH_DEV ? 7 : 0>(g, cv, odd, s, k, cf, pe, pmx, pmy, pmz, nacc);
}

// Hides v from the optimizer's value tracking, keeping only that it is non-negative.
__device__ __forceinline__ void opaque_nonneg(int &v)
{
    asm volatile("" : "+v"(v));
    v &= 0x7FFFFFFF;
}

// Geometry of one column (fixed j and y) of colour c: everything but z.
struct Column {
    int hcol;    // j + (L/2) y
    int idcol;   // 2 j + L y
    int par;     // (y + c) & 1: x-parity is (par + z) & 1
    int dxm0;    // x-1 neighbour minus h when the x-parity is 0 (else 0)
    int dxp1;    // x+1 neighbour minus h when the x-parity is 1 (else 0)
    int dym, dyp;
};

__device__ __forceinline__ Column make_column(int L, int col, int c)
{
    const int HL = L >> 1;
    const int j = col % HL, y = col / HL;
    Column k;
    k.hcol = col;
    k.idcol = 2 * j + L * y;
    k.par = (y + c) & 1;
    k.dxm0 = (j == 0) ? HL - 1 : -1;
    k.dxp1 = (j == HL - 1) ? -(HL - 1) : 1;
    k.dym = (y == 0) ? (L - 1) * HL : -HL;
    k.dyp = (y == L - 1) ? -(L - 1) * HL : HL;
    return k;
}

// Site z of a column; dzm / dzp: half-index offsets of the z-1 / z+1 neighbours (they differ
// from -plane / +plane only on the wrap-around planes).
template <int L>
__device__ __forceinline__ Site column_site(const Column &k, int z, int dzm, int dzp)
{
    constexpr int PLANE = L * L / 2;
    Site s;
    const int p = (k.par + z) & 1;
    s.h = k.hcol + PLANE * z;
    s.id = k.idcol + p + L * L * z;
    s.nb[0] = s.h + (p ? 0 : k.dxm0);
    s.nb[1] = s.h + (p ? k.dxp1 : 0);
    s.nb[2] = s.h + k.dym;
    s.nb[3] = s.h + k.dyp;
    s.nb[4] = s.h + dzm;
    s.nb[5] = s.h + dzp;
    return s;
}

// Colour- and sweep-independent site geometry of a lane in the column map with few sites
// per lane (G >= plane, NZ <= 8), computed once per launch. Half-indices are those of the
// lane's first site (t = 0); site t adds the compile-time offset plane * DZ * t.
struct LaneGeom {
    bool owns;             // lane < DZ * plane
    int z0, zlast;
    int b_own, b_ym, b_yp;  // own and y-neighbour half-indices
    int b_zm, b_zp;         // z-1 neighbour of the first site, z+1 neighbour of the last (wrap-aware)
    int dxm0, dxp1;         // x-1 offset when the x-parity is 0, x+1 offset when it is 1
    int par0;               // x-parity of the first site for colour 0
    int id00;               // site id of the first site for colour 0, less its x-parity
};

template <int LC, int G>
struct ColzShape {
    static constexpr int PLANE = LC * LC / 2;
    static constexpr bool WIDE = LC != 0 && G >= PLANE;
    static constexpr int DZ = WIDE ? G / PLANE : 1;
    static constexpr int NZ = WIDE ? (LC + DZ - 1) / DZ : 0;
    static constexpr bool FEW = WIDE && NZ <= 8;  // geometry kept in registers across sweeps
};

template <int LC, int G>
__device__ __forceinline__ LaneGeom make_lane_geom(int lane)
{
    using S = ColzShape<LC, G>;
    constexpr int PLANE = S::PLANE, DZ = S::DZ, NZ = S::NZ, HL = LC / 2;
    LaneGeom q;
    q.owns = lane < DZ * PLANE;
    const int col = lane % PLANE, j = col % HL, y = col / HL;
    q.z0 = lane / PLANE;
    q.zlast = q.z0 + DZ * (NZ - 1);
    q.b_own = col + PLANE * q.z0;
    q.b_ym = q.b_own + ((y == 0) ? (LC - 1) * HL : -HL);
    q.b_yp = q.b_own + ((y == LC - 1) ? -(LC - 1) * HL : HL);
    q.b_zm = q.b_own + ((q.z0 == 0) ? (LC - 1) * PLANE : -PLANE);
    q.b_zp = q.b_own + DZ * (NZ - 1) * PLANE + ((q.zlast == LC - 1) ? -(LC - 1) * PLANE : PLANE);
    q.dxm0 = (j == 0) ? HL - 1 : -1;
    q.dxp1 = (j == HL - 1) ? -(HL - 1) : 1;
    q.par0 = (y + q.z0) & 1;
    q.id00 = 2 * j + LC * y + LC * LC * q.z0;
    opaque_nonneg(q.b_own);
    opaque_nonneg(q.b_ym);
    opaque_nonneg(q.b_yp);
    opaque_nonneg(q.b_zm);
    opaque_nonneg(q.b_zp);
    return q;
}

// One half-sweep (colour c) of this lane's sites.
//   COLZ (compile-time L): a lane owns whole columns (fixed x-pair and y) and a stride of z;
//   for G >= plane (plane = L^2/2 sites of a colour) lane = column + plane z0 and
//   z = z0 + DZ t with DZ = G / plane, else the lane owns columns lane + G t and every z
//   (the wrap-around planes z = 0 and L-1 peeled off).
//   FLAT (any L): lane owns half-indices lane + G s.
template <typename T, int LC, int G, int MAP, int PL>
__device__ __forceinline__ void half_sweep(const GroupCtx<T> &g, const LaneGeom &q, int c, uint32_t k,
                                           const Coef<T> &cf, T &pe, T &pmx, T &pmy, T &pmz,
                                           unsigned long long &nacc)
{
    const int L = LC ? LC : g.L;
    const int HALF = L * L * L / 2;
    // (c is a constant after inlining, so each colour's address space is known statically;
    // colour 1 follows colour 0 unless the colours are split between LDS and device memory)
    constexpr bool SPLIT = PL == PL_SPLIT || PL == PL_SPLIT_XY, MEM = PL == PL_MEM, XY = PL == PL_SPLIT_XY;
    // components in device memory (bit 0: x, 1: y, 2: z) of colour 0 and colour 1
    constexpr int DEV0 = MEM ? 7 : (XY ? 4 : 0), DEV1 = (MEM || SPLIT) ? 7 : 0;
    T *const sp1 = SPLIT ? g.sp1 : g.sp + 3 * HALF;
    T *const c0[3] = {g.sp, g.sp + HALF, XY ? g.sp0z : g.sp + 2 * HALF};
    T *const c1[3] = {sp1, sp1 + HALF, sp1 + 2 * HALF};
    const ColourView<T> cv = c ? ColourView<T>{{c1[0], c1[1], c1[2]}, {c0[0], c0[1], c0[2]}}
                               : ColourView<T>{{c0[0], c0[1], c0[2]}, {c1[0], c1[1], c1[2]}};
    const bool odd = c != 0;
    // The lane's site geometry and the sweep-independent part of its counters are cheap to
    // recompute here; an opaque lane index keeps the compiler from hoisting them for all of
    // the lane's sites out of the sweep loop, which would cost more registers (occupancy,
    // spills) than it saves.
    int lane = g.lane;
    asm volatile("" : "+v"(lane));
    // ... but its range stays known (non-negative bases let the backend fold the constant
    // parts of the LDS addresses into the instructions' offset fields)
    if constexpr ((G & (G - 1)) == 0) lane &= G - 1;
    else __builtin_assume(lane >= 0 && lane < G);
    auto up = [&](const Site &s) {
        if (odd) update_site_v<T, false, DEV1, DEV0>(g, cv, odd, s, k, cf, pe, pmx, pmy, pmz, nacc);
        else update_site_v<T, false, DEV0, DEV1>(g, cv, odd, s, k, cf, pe, pmx, pmy, pmz, nacc);
    };
    if constexpr (MAP == COLZ && LC != 0) {
        constexpr int PLANE = LC * LC / 2;
        if constexpr (G >= PLANE) {
            constexpr int DZ = G / PLANE;
            constexpr int NZ = (LC + DZ - 1) / DZ;
            if constexpr (NZ > 8) {
                if (lane >= DZ * PLANE) return;
                const int z0 = lane / PLANE;
                const Column col = make_column(LC, lane % PLANE, c);
                // many sites per lane: a rolled loop (the wrap planes peeled)
                const int zlast = z0 + DZ * (NZ - 1);
                const int dzm0 = (z0 == 0) ? (LC - 1) * PLANE : -PLANE;
                const int dzpl = (zlast == LC - 1) ? -(LC - 1) * PLANE : PLANE;
                up(column_site<LC>(col, z0, dzm0, PLANE));
#pragma unroll 2
                for (int t = 1; t < NZ - 1; ++t) up(column_site<LC>(col, z0 + DZ * t, -PLANE, PLANE));
                if ((LC % DZ) == 0 || zlast < LC) up(column_site<LC>(col, zlast, -PLANE, dzpl));
                return;
            }
            // (uniform when every lane owns sites: the wave's accept count stays scalar)
            if constexpr (DZ * PLANE < G) {
                if (!q.owns) return;
            }
            // Colour-dependent part: the x-parity of the first site and the x-neighbours; the
            // rest of the geometry comes from q. Opaque per half-sweep so that the counters'
            // sweep-independent Philox work is not hoisted for all of the lane's sites.
            const int p0 = q.par0 ^ c;
            int b_xm0 = q.b_own + (p0 ? 0 : q.dxm0), b_xp0 = q.b_own + (p0 ? q.dxp1 : 0);
            int b_xm1 = q.b_own + (p0 ? q.dxm0 : 0), b_xp1 = q.b_own + (p0 ? 0 : q.dxp1);
            int id0 = q.id00 + p0;
            opaque_nonneg(b_xm0);
            opaque_nonneg(b_xp0);
            opaque_nonneg(id0);
            if constexpr (DZ & 1) {
                opaque_nonneg(b_xm1);
                opaque_nonneg(b_xp1);
            }
#pragma unroll
            for (int t = 0; t < (NZ > 8 ? 1 : NZ); ++t) {
                const int o = PLANE * DZ * t;
                const bool flip = (DZ & 1) && (t & 1);
                Site s;
                s.h = q.b_own + o;
                s.id = id0 + LC * LC * DZ * t + (flip ? (p0 ? -1 : 1) : 0);
                s.nb[0] = (flip ? b_xm1 : b_xm0) + o;
                s.nb[1] = (flip ? b_xp1 : b_xp0) + o;
                s.nb[2] = q.b_ym + o;
                s.nb[3] = q.b_yp + o;
                s.nb[4] = t == 0 ? q.b_zm : q.b_own + o - PLANE;
                s.nb[5] = t == NZ - 1 ? q.b_zp : q.b_own + o + PLANE;
                if ((LC % DZ) == 0 || t < NZ - 1 || q.zlast < LC) up(s);
            }
        } else {
            constexpr int NCOL = (PLANE + G - 1) / G;
#pragma unroll 1
            for (int cc = 0; cc < NCOL; ++cc) {
                const int ci = lane + G * cc;
                if ((PLANE % G) != 0 && ci >= PLANE) break;
                const Column col = make_column(LC, ci, c);
                up(column_site<LC>(col, 0, (LC - 1) * PLANE, PLANE));
#pragma unroll 2
                for (int z = 1; z < LC - 1; ++z) up(column_site<LC>(col, z, -PLANE, PLANE));
                up(column_site<LC>(col, LC - 1, -PLANE, -(LC - 1) * PLANE));
            }
        }
    } else {
        const int SPL = (HALF + G - 1) / G;
#pragma unroll 2
        for (int s = 0; s < SPL; ++s) {
            const int h = lane + G * s;
            if (h < HALF) up(flat_site(L, h, c));
        }
    }
}

// Initial state of Sec. 2.2 (Philox counter (id, 0, path, TAG_INIT)): the group's lanes take
// the path's sites in a flat stride. sp0 / sp1: colour-0 / colour-1 spins (sp1 null: colour 1
// follows colour 0); sp0z: colour 0's z components when they are apart from its x and y (else
// null). Out of line (runs once): inlined, it crashes the ROCm 7.2 optimizer (SimplifyCFG).
template <typename T, int G>
__device__ __attribute__((noinline)) void init_path(T *sp0, T *sp1, T *sp0z, int L, int lane, uint32_t path,
                                                    uint32_t key0, uint32_t key1, uint32_t ctr3, int init)
{
    const int HALF = L * L * L / 2;
    // mixed start: even paths from the random (sphere) start, odd paths ordered
    if (init == INIT_MIXED) init = (path & 1u) ? INIT_ORDERED : INIT_SPHERE;
    for (int t = lane; t < 2 * HALF; t += G) {
        const int c = t >= HALF, h = t - c * HALF;
        const Site s = flat_site(L, h, c);
        T x, y, z;
        if (init == INIT_ORDERED) {
            x = T(0);
            y = T(0);
            z = T(1);
        } else {
            const Words w = philox4x32_10((uint32_t)s.id, 0u, path, TAG_INIT | ctr3, key0, key1);
            if (init == INIT_ANGLES) Arith<T>::angles(w.w0, w.w1, x, y, z);
            else Arith<T>::sphere(w.w0, w.w1, x, y, z);
        }
        T *own = c ? (sp1 ? sp1 : sp0 + 3 * HALF) : sp0;
        T *ownz = (!c && sp0z) ? sp0z : own + 2 * HALF;
        own[h] = x;
        own[HALF + h] = y;
        ownz[h] = z;
    }
}

// FP32 only: S <- S / |S| for every site of the path (each site touched by one lane; sp0, sp1
// and sp0z as for init_path). Out of line (runs every renorm_every sweeps): inlined, it
// crashes the ROCm 7.2 optimizer (SimplifyCFG).
template <int G>
__device__ __attribute__((noinline)) void renorm_path(float *sp0, float *sp1, float *sp0z, int L, int lane)
{
    const int HALF = L * L * L / 2;
    for (int t = lane; t < 2 * HALF; t += G) {
        const int c = t >= HALF, h = t - c * HALF;
        float *own = c ? (sp1 ? sp1 : sp0 + 3 * HALF) : sp0;
        float *ownz = (!c && sp0z) ? sp0z : own + 2 * HALF;
        const float x = own[h], y = own[HALF + h], z = ownz[h];
        const float r = __builtin_amdgcn_rsqf(fmaf(z, z, fmaf(y, y, x * x)));
        own[h] = x * r;
        own[HALF + h] = y * r;
        ownz[h] = z * r;
    }
}

// Sweeps [k0, k1) of one path group. All groups of the workgroup call this together (same
// instance and sweep range), so __syncthreads() separates the half-sweeps of all of them.
// Idle groups (path >= n_paths) and idle lanes still take every barrier.
template <typename T, int LC, int G, int MAP, int PL>
__device__ __forceinline__ void path_sweeps(const GroupCtx<T> &g, const InstDev &in, int k0, int k1, bool fresh)
{
    const int L = LC ? LC : g.L;
    const double Nd = (double)L * L * L;
    const int n_therm = in.n_therm, trace_sweeps = in.trace_sweeps, renorm_every = in.renorm_every;
    const double J = in.J;
    double *const trace = in.trace;
    Coef<T> cf;
    cf.beta = (T)in.beta;
    cf.J = (T)in.J;
    cf.q = (float)(in.beta * in.J * 1.4426950408889634);  // beta J log2(e)
    const int wave = g.lane >> 6;
    constexpr int W = G / 64;  // waves per path group
    unsigned long long nacc = 0;  // this wave's accepted moves

    // colour-1 spins and colour-0 z components when they do not follow colour 0's x and y
    T *const sp1 = (PL == PL_SPLIT || PL == PL_SPLIT_XY) ? g.sp1 : nullptr;
    T *const sp0z = PL == PL_SPLIT_XY ? g.sp0z : nullptr;
    if (g.active && fresh) init_path<T, G>(g.sp, sp1, sp0z, L, g.lane, g.path, g.key0, g.key1, g.ctr3, in.init);
    __syncthreads();
    LaneGeom geom{};
    if constexpr (MAP == COLZ && ColzShape<LC, G>::FEW) {
        int lane = g.lane;
        asm volatile("" : "+v"(lane));  // not hoisted out of a persistent kernel's item loop
        geom = make_lane_geom<LC, G>(lane);
    }

    for (int k = k0; k < k1; ++k) {
        if constexpr (std::is_same<T, float>::value) {
            if (renorm_every > 0 && k > 0 && k % renorm_every == 0) {
                if (g.active) renorm_path<G>(g.sp, sp1, sp0z, L, g.lane);
                __syncthreads();
            }
        }
        T pe = T(0), pmx = T(0), pmy = T(0), pmz = T(0);
        if (g.active) half_sweep<T, LC, G, MAP, PL>(g, geom, 0, (uint32_t)k, cf, pe, pmx, pmy, pmz, nacc);
        __syncthreads();
        if (g.active) half_sweep<T, LC, G, MAP, PL>(g, geom, 1, (uint32_t)k, cf, pe, pmx, pmy, pmz, nacc);
        const bool meas = k >= n_therm || k < trace_sweeps || k == k1 - 1;
        if (meas) {
            // sums over each 16-lane row; one lane per row leaves its row's four partials
            pe = row_sum(pe);
            pmx = row_sum(pmx);
            pmy = row_sum(pmy);
            pmz = row_sum(pmz);
            if ((g.lane & 15) == 0) {
                T *slot = g.red + 4 * (g.lane >> 4);
                slot[0] = pe;
                slot[1] = pmx;
                slot[2] = pmy;
                slot[3] = pmz;
            }
        }
        __syncthreads();
        if (meas && g.active && wave == 0) {
            // the group's first wave adds up the row partials (one row per lane)
            T se = T(0), sx = T(0), sy = T(0), sz = T(0);
            if (g.lane < 4 * W) {
                se = g.red[4 * g.lane + 0];
                sx = g.red[4 * g.lane + 1];
                sy = g.red[4 * g.lane + 2];
                sz = g.red[4 * g.lane + 3];
            }
            se = wave_sum(se);
            sx = wave_sum(sx);
            sy = wave_sum(sy);
            sz = wave_sum(sz);
            if (g.lane == 0) {
                // Every bond joins an even and an odd site: E = -J sum_odd S_i . h_i.
                const double e = -J * (double)se / Nd;
                const double mx = (double)sx / Nd, my = (double)sy / Nd, mz = (double)sz / Nd;
                if (k >= n_therm) {
                    const double m = sqrt(mx * mx + my * my + mz * mz);
                    g.shacc[0] += e;
                    g.shacc[1] += e * e;
                    g.shacc[2] += m;
                    g.shacc[3] += m * m;
                    g.shacc[4] += (m * m) * (m * m);
                }
                if (k < trace_sweeps) {
                    double *tr = trace + ((size_t)g.path * trace_sweeps + k) * 4;
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
    }
    if (g.active && (g.lane & 63) == 0) atomicAdd((unsigned long long *)&g.shacc[9], nacc);
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

// ------------------------------------------------------------------ colour-split z-plane ring
// For lattices too large for LDS whose z-planes are not (L = 48 in FP32): the path's spins
// stay in device memory and the workgroup (one path, B lanes) sweeps them through a ring of
// RING = 5 plane slots in LDS, each slot holding one z-plane's colour-0 and colour-1 halves
// (three components each). One pass is one sweep, in L + 3 steps with one barrier each:
//   stage 0 (colour 0) updates virtual plane tau at step tau, 0 <= tau < L;
//   stage 1 (colour 1) updates virtual plane tau - 2 at step tau, 3 <= tau <= L + 2, i.e. the
//   virtual planes 1 .. L, so physical plane 0 comes last, after colour 0's plane L - 1.
// A colour-1 update at plane v reads colour 0 of planes v - 1 .. v + 1, all updated in earlier
// steps; a colour-0 update at plane v reads colour 1 of planes v - 1 .. v + 1, none of which
// is updated before step v + 1 (plane 0's wrap-around neighbour L - 1 last of all): each site
// sees exactly the neighbour values of the sequential half-sweep order. The two stages of a
// step touch disjoint data. Virtual plane v lives in slot v mod RING: colour 0 of plane v is
// in the ring during steps v .. v + 3, colour 1 during steps v - 1 .. v + 2, and each step
// brings in the next step's two half-planes (colour 0 of plane tau + 1, colour 1 of plane
// tau + 2), loaded into registers at the start of the step and stored into the ring at its
// end, into slots whose previous half-planes are no longer read. Every update writes its
// outcome straight to device memory (only the accepted ones, except on renormalisation
// passes); colour 0 also updates its ring copy, which colour 1 reads later, and the two
// colour-0 planes read again as virtual planes L and L + 1 are reloaded from device memory.
// Device-memory traffic per update: 12 (2L + 4) / (2L) B read + 12 B written, 24.5 B at L = 48.
// Renormalisation (FP32, every renorm_every sweeps) happens on load: every site is normalised
// when its plane first enters the ring in the pass (colour 0 virtual planes 0 .. L - 1, every
// colour-1 load) and written back whether or not its move is accepted, which leaves the spins
// bit-identical to the other kernels'.
// Half ring (PL_HRING, for sides whose two-colour slots do not fit: L = 64 in FP32): colour 1
// is updated in place in device memory; the LDS holds HR_SLOTS = 4 slots of colour 0 and two
// buffers of colour 1 (the plane being updated and the one below). Each step has two phases,
// each over every lane (path_sweeps_hring): colour 0 of plane tau reads five of its six
// neighbours from the buffers and the one above from device memory, then colour 1 of plane
// tau - 1 reads all its neighbours from the slots. A colour-1 plane is read from device memory
// twice per pass, one step apart (into its buffer with the plane below, and for its own
// update), so the L2 still holds it the second time. Renormalisation passes normalise colour
// 1 in place before the pass (the colour-0 rule as above).
// Two-sweep ring (PL_RING2, L = 32 and 48 in FP32): two sweeps ks, ks + 1 per pass, as four
// stages: stage 0 (colour 0 of sweep ks) at virtual plane tau, stage 1 (colour 1, ks) at
// tau - 1, stage 2 (colour 0, ks + 1) at tau - 3, stage 3 (colour 1, ks + 1) at tau - 4, stage
// j over virtual planes j .. j + L - 1 (each starts one plane further round the periodic
// z-ring, so physical planes 0 .. j - 1 come last for it). A step has two phases with a barrier
// after each: stages 0 and 2 (colour 0), then stages 1 and 3 (colour 1); the stages of a phase
// touch disjoint planes, and each update sees exactly the neighbour values of the sequential
// half-sweep order. The LDS holds R2_SLOTS0 = 5 colour-0 slots (plane v in slot v mod 5 during
// steps v .. v + 4) and R2_SLOTS1 = 6 colour-1 slots (plane v in slot v mod 6 during steps
// v - 1 .. v + 4), 152 KB at L = 48; every neighbour comes from LDS or registers:
//   stage 0 takes its own spins from registers (loaded from device memory the step before)
//   and writes every outcome into its slot, whose previous plane v - 5 was written back to
//   device memory a step earlier;
//   stage 3 takes its own spins from registers, copied from their slot in phase 1 (before
//   phase 2 stores colour 1 of plane tau + 2 over them), and its neighbours below (colour 0 of
//   plane v - 1) from registers copied from their slot in phase 2 of the step before (that
//   slot takes colour 0 of plane tau in phase 1), and writes every outcome to device memory;
//   colour 0 of plane v is written back at step v + 4, after stage 2's update at step v + 3;
//   colour 1 reaches device memory from stage 3, and from stage 1 for virtual planes 1 and 2,
//   whose sweep-ks state stage 3 reads again as virtual planes L + 1 and L + 2;
//   the virtual planes past L - 1 are reloaded from device memory (colour 0 of L .. L + 3,
//   copied into their slots by the lanes of stage 0; colour 1 of L .. L + 2).
// Device-memory traffic per update: about 12 (1 + 3/L) B (each colour-plane read and written
// once per two sweeps, plus the wrap-around reloads): 12.75 B at L = 48 instead of 24.5.
// A one-sweep pass (the last sweep of an odd count, or a sweep before a renormalisation
// boundary) runs stages 0 and 1 alone, which then write their outcomes to device memory
// directly. Renormalisation passes normalise the whole lattice in place first. In a phase,
// the active stages' sites (a plane of each) are dealt to the lanes as u = lane + B i, stage
// u / plane, site u mod plane: wave-uniform, since the plane and B are multiples of 64, and
// a phase with one active stage gives it every lane.
constexpr int RING = 5;

// The half ring's LDS: HR_SLOTS slots of colour 0 and two buffers of colour 1.
constexpr int HR_SLOTS = 4;

// The two-sweep ring's LDS: R2_SLOTS0 slots of colour 0, then R2_SLOTS1 of colour 1.
constexpr int R2_SLOTS0 = 5, R2_SLOTS1 = 6;

// LDS of a ring workgroup: the plane slots (RING of both colours of a z-plane; half ring:
// HR_SLOTS of colour 0 and two colour-1 buffers), accumulators, reduction slots.
template <typename T>
__host__ __device__ constexpr size_t ring_lds_bytes(int L, int B, int pl)
{
    const int halves = pl == PL_HRING ? HR_SLOTS + 2 : pl == PL_RING2 ? R2_SLOTS0 + R2_SLOTS1 : 2 * RING;
    return (size_t)halves * 3 * ((size_t)L * L / 2) * sizeof(T) + 128 + (size_t)(B / 16) * 4 * sizeof(T);
}

// LDS bytes of one workgroup: spins (all of them, or colour 0), accumulators, reduction
// slots (four partials per 16-lane row).
template <typename T>
__host__ __device__ constexpr size_t lds_layout_bytes(int L, int B, int G, int pl)
{
    if (pl == PL_RING || pl == PL_HRING || pl == PL_RING2) return ring_lds_bytes<T>(L, B, pl);
    const size_t ns = 3 * (size_t)L * L * L * sizeof(T);
    return (size_t)(B / G) * (pl == PL_LDS ? ns : pl == PL_SPLIT ? ns / 2 : pl == PL_SPLIT_XY ? ns / 3 : 0) +
           (size_t)(B / G) * 128 +
           (size_t)(B / 16) * 4 * sizeof(T);
}

// Half-planes in flight between device memory and the ring: lane t holds groups of E
// consecutive sites (one 16-byte vector per component: E = 4 in FP32, 2 in FP64)
// q = t + B i of two half-planes, q < PLANE / E in the first, the rest in the second.
template <typename T, int LC, int B>
struct RingRegs {
    using V = typename std::conditional<std::is_same<T, float>::value, float4, double2>::type;
    static constexpr int E = 16 / (int)sizeof(T);
    static constexpr int PLANE = LC * LC / 2, NQ = PLANE / E, R = (2 * NQ + B - 1) / B;
    V x[R], y[R], z[R];
};

template <typename V, typename T>
__device__ __forceinline__ V ld16(const T *base, uint32_t byte_off)
{
    return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) + byte_off);
}

__device__ __forceinline__ void normalise_sites(float4 &x, float4 &y, float4 &z)
{
    const float ra = __builtin_amdgcn_rsqf(fmaf(z.x, z.x, fmaf(y.x, y.x, x.x * x.x)));
    const float rb = __builtin_amdgcn_rsqf(fmaf(z.y, z.y, fmaf(y.y, y.y, x.y * x.y)));
    const float rc = __builtin_amdgcn_rsqf(fmaf(z.z, z.z, fmaf(y.z, y.z, x.z * x.z)));
    const float rd = __builtin_amdgcn_rsqf(fmaf(z.w, z.w, fmaf(y.w, y.w, x.w * x.w)));
    x = make_float4(x.x * ra, x.y * rb, x.z * rc, x.w * rd);
    y = make_float4(y.x * ra, y.y * rb, y.z * rc, y.w * rd);
    z = make_float4(z.x * ra, z.y * rb, z.z * rc, z.w * rd);
}

__device__ __forceinline__ void normalise_sites(double2 &, double2 &, double2 &) {}  // FP64: never

// Loads colour c0 of plane zp0 (when h0) and colour c1 of plane zp1 (when h1) from the path's
// device-memory spins gsp into registers.
template <typename T, int LC, int B>
__device__ __forceinline__ void ring_load(RingRegs<T, LC, B> &r, const T *gsp, int c0, int zp0, bool h0, int c1,
                                          int zp1, bool h1, int tid)
{
    using R = RingRegs<T, LC, B>;
    using V = typename R::V;
    constexpr int PLANE = R::PLANE, NQ = R::NQ, E = R::E, HALF = LC * PLANE;
    constexpr uint32_t CB = HALF * sizeof(T);  // bytes between components
#pragma unroll
    for (int i = 0; i < R::R; ++i) {
        const int q = tid + B * i;
        const bool second = q >= NQ;
        if (q < 2 * NQ && (second ? h1 : h0)) {
            const int c = second ? c1 : c0, zp = second ? zp1 : zp0, rq = q - (second ? NQ : 0);
            const uint32_t off = (uint32_t)(c * 3 * HALF + zp * PLANE + E * rq) * (uint32_t)sizeof(T);
            r.x[i] = ld16<V>(gsp, off);
            r.y[i] = ld16<V>(gsp, off + CB);
            r.z[i] = ld16<V>(gsp, off + 2u * CB);
        }
    }
}

// Stores what ring_load brought in into ring slots s0 / s1 (normalising first where n0 / n1).
// HR (half ring): the slots hold colour 0 only, and the second half-plane (colour 1) goes to
// colour-1 buffer s1 after the HR_SLOTS slots (c1 unused).
template <typename T, int LC, int B, bool HR = false>
__device__ __forceinline__ void ring_store(RingRegs<T, LC, B> &r, T *ring, int c0, int s0, bool h0, bool n0, int c1,
                                           int s1, bool h1, bool n1, int tid)
{
    using R = RingRegs<T, LC, B>;
    using V = typename R::V;
    constexpr int PLANE = R::PLANE, NQ = R::NQ, E = R::E, SLOT = (HR ? 3 : 6) * PLANE;
#pragma unroll
    for (int i = 0; i < R::R; ++i) {
        const int q = tid + B * i;
        const bool second = q >= NQ;
        if (q < 2 * NQ && (second ? h1 : h0)) {
            const int c = second ? c1 : c0, sl = second ? s1 : s0, rq = q - (second ? NQ : 0);
            if (second ? n1 : n0) normalise_sites(r.x[i], r.y[i], r.z[i]);
            T *o = (HR && second) ? ring + HR_SLOTS * SLOT + sl * 3 * PLANE + E * rq
                                  : ring + sl * SLOT + c * 3 * PLANE + E * rq;
            *reinterpret_cast<V *>(o) = r.x[i];
            *reinterpret_cast<V *>(o + PLANE) = r.y[i];
            *reinterpret_cast<V *>(o + 2 * PLANE) = r.z[i];
        }
    }
}

// Geometry of the sites a lane updates in every plane: in-plane half-index s = rank 64 + wl +
// (B/2) t, its site id less the x-parity and the z part, the parity of y, and the in-plane
// neighbour offsets (x-1 when the x-parity is 0, x+1 when it is 1, y-1, y+1).
struct RingSite {
    int s, idb, ypar, xm0, xp1, ym, yp, y;
};

// With (B/2) a multiple of the row length L/2 a lane's sites share their x position and are
// (B/2)/(L/2) rows apart, so only the first site's geometry is kept (fewer registers).
template <int LC, int B>
constexpr bool ring_compact() { return ((B / 2) % (LC / 2)) == 0; }

template <typename T, int C, int LC, int B, int K>
__device__ __forceinline__ void ring_stage(const GroupCtx<T> &g, const RingSite (&q)[K], T *ring, T *gsp, int v,
                                           uint32_t k, const Coef<T> &cf, bool rn, T &pe, T &pmx, T &pmy, T &pmz,
                                           unsigned long long &nacc)
{
    constexpr int PLANE = LC * LC / 2, HALF = LC * PLANE, SLOT = 6 * PLANE, SL = B / 2;
    const int zp = v < LC ? v : v - LC;
    const int sl = v % RING;
    const int rdm = ((v + RING - 1) % RING - sl) * SLOT, rdp = ((v + 1) % RING - sl) * SLOT;
    T *const own = ring + sl * SLOT + C * 3 * PLANE;
    const T *const oth = ring + sl * SLOT + (1 - C) * 3 * PLANE;
    const ColourView<T> cv{{own, own + PLANE, own + 2 * PLANE}, {oth, oth + PLANE, oth + 2 * PLANE}};
    T *const gx = gsp + C * 3 * HALF + zp * PLANE, *const gy = gx + HALF, *const gz = gx + 2 * HALF;
    const int zpar = zp & 1, idz = LC * LC * zp;
    constexpr bool COMPACT = ring_compact<LC, B>();
    constexpr int HL = LC / 2, DY = COMPACT ? SL / HL : 0;
    auto site = [&](int t) {
        RingSite r;
        if constexpr (COMPACT) {
            // sites t of a lane: DY t rows below its first one, same x
            r.s = q[0].s + SL * t;
            r.y = q[0].y + DY * t;
            r.idb = q[0].idb + LC * DY * t;
            r.ypar = (q[0].ypar + DY * t) & 1;
            r.xm0 = q[0].xm0;
            r.xp1 = q[0].xp1;
            r.ym = (r.y == 0) ? (LC - 1) * HL : -HL;
            r.yp = (r.y == LC - 1) ? -(LC - 1) * HL : HL;
        } else {
            r = q[t];
        }
        if ((PLANE % SL) == 0 || t < K - 1 || r.s < PLANE) {
            const int p = (r.ypar + zpar + C) & 1;
            const int h = r.s;  // in-plane half-index
            Site st;
            st.h = h;
            st.id = r.idb + p + idz;
            st.nb[0] = h + (p ? 0 : r.xm0);
            st.nb[1] = h + (p ? r.xp1 : 0);
            st.nb[2] = h + r.ym;
            st.nb[3] = h + r.yp;
            st.nb[4] = h + rdm;
            st.nb[5] = h + rdp;
            update_site_s<T, false, 0, 0>(g, cv, C != 0, st, k, cf, pe, pmx, pmy, pmz, nacc,
                                          [&](bool acc, T nx, T ny, T nz, T sx, T sy, T sz) {
                                              if (C == 0 && acc) {
                                                  own[h] = nx;
                                                  own[PLANE + h] = ny;
                                                  own[2 * PLANE + h] = nz;
                                              }
                                              if (acc || rn) {
                                                  spin_at<true>(gx, h) = acc ? nx : sx;
                                                  spin_at<true>(gy, h) = acc ? ny : sy;
                                                  spin_at<true>(gz, h) = acc ? nz : sz;
                                              }
                                          });
        }
    };
    if constexpr (COMPACT) {
        // (rolled: the sites' geometry comes from the first one, and one update at a time keeps
        // the registers of a 1024-lane workgroup within budget)
#pragma unroll 1
        for (int t = 0; t < K; ++t) site(t);
    } else {
#pragma unroll
        for (int t = 0; t < K; ++t) site(t);
    }
}

// One phase of the half ring: colour C of virtual plane v, every lane of the workgroup with
// K sites q of the plane. Colour 0 (own in its slot) reads colour 1 in-plane from the buffer of
// plane v, below from the buffer of plane v - 1 and above from device memory; colour 1 takes
// its own spins from own1 (read from the plane's buffer before the phase) and colour 0 of
// planes v - 1 .. v + 1 from their slots. Outcomes go to device memory (colour 0 also to its
// slot); colour 1 is normalised in place before a renormalisation pass, colour 0 on its way
// into the ring.
template <typename T, int C, int LC, int B, int K>
__device__ __forceinline__ void hring_stage(const GroupCtx<T> &g, const RingSite (&q)[K], const T (&own1)[K][3], T *ring,
                                            T *gsp, int v, uint32_t k, const Coef<T> &cf, bool rn, T &pe, T &pmx,
                                            T &pmy, T &pmz, unsigned long long &nacc)
{
    constexpr int PLANE = LC * LC / 2, HALF = LC * PLANE, SLOT = 3 * PLANE;
    const int zp = v < LC ? v : v - LC;
    const int zpar = zp & 1, idz = LC * LC * zp;
    // colour 1 in device memory, indexed from each component's start (non-negative indices):
    // zb / zbp the first sites of plane zp and of the plane above
    T *const gc1 = gsp + 3 * HALF;
    const int zb = zp * PLANE, zbp = (zp == LC - 1 ? 0 : zp + 1) * PLANE;
    T *const g0 = gsp + zp * PLANE;  // colour 0 of plane zp in device memory (components HALF apart)
    T *const s0 = ring + (v % HR_SLOTS) * SLOT;  // colour 0 of plane v
    const T *const sm = ring + ((v + HR_SLOTS - 1) % HR_SLOTS) * SLOT, *const sp = ring + ((v + 1) % HR_SLOTS) * SLOT;
    const T *const b0 = ring + HR_SLOTS * SLOT + (v & 1) * SLOT;        // colour 1 of plane v
    const T *const bm = ring + HR_SLOTS * SLOT + ((v + 1) & 1) * SLOT;  // colour 1 of plane v - 1
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const RingSite &r = q[t];
        if ((PLANE % B) == 0 || t < K - 1 || r.s < PLANE) {
            const int p = (r.ypar + zpar + C) & 1;
            const int h = r.s;  // in-plane half-index
            Site st;
            st.h = h;
            st.id = r.idb + p + idz;
            // in-plane neighbours (plane-local indices); the z-neighbours share h
            st.nb[0] = h + (p ? 0 : r.xm0);
            st.nb[1] = h + (p ? r.xp1 : 0);
            st.nb[2] = h + r.ym;
            st.nb[3] = h + r.yp;
            st.nb[4] = st.nb[5] = h;
            if constexpr (C == 0) {
                update_site_f<T, false>(
                    g, false, st, k, cf, pe, pmx, pmy, pmz, nacc, [&](int c) { return s0[c * PLANE + h]; },
                    [&](int c, int n) {
                        return n < 4    ? b0[c * PLANE + st.nb[n]]
                               : n == 4 ? bm[c * PLANE + h]
                                        : spin_at<true>(gc1 + c * HALF, zbp + h);
                    },
                    [&](bool acc, T nx, T ny, T nz, T sx, T sy, T sz) {
                        if (acc) {
                            s0[h] = nx;
                            s0[PLANE + h] = ny;
                            s0[2 * PLANE + h] = nz;
                        }
                        if (acc || rn) {
                            spin_at<true>(g0, h) = acc ? nx : sx;
                            spin_at<true>(g0 + HALF, h) = acc ? ny : sy;
                            spin_at<true>(g0 + 2 * HALF, h) = acc ? nz : sz;
                        }
                    });
            } else {
                update_site_f<T, false>(
                    g, true, st, k, cf, pe, pmx, pmy, pmz, nacc, [&](int c) { return own1[t][c]; },
                    [&](int c, int n) {
                        return n < 4 ? s0[c * PLANE + st.nb[n]] : n == 4 ? sm[c * PLANE + h] : sp[c * PLANE + h];
                    },
                    [&](bool acc, T nx, T ny, T nz, T, T, T) {
                        if (acc) {
                            spin_at<true>(gc1, zb + h) = nx;
                            spin_at<true>(gc1 + HALF, zb + h) = ny;
                            spin_at<true>(gc1 + 2 * HALF, zb + h) = nz;
                        }
                    });
            }
        }
    }
}

// Measurement of sweep ks of a ring pass (the state after it; every site was added once to the
// lane partials pe, pmx, pmy, pmz): 16-lane row sums into the reduction slots, then wave 0 sums
// them and adds the sweep's e and m to the path's accumulators and trace.
template <typename T, int W>
__device__ __forceinline__ void ring_measure(const GroupCtx<T> &g, const InstDev &in, int ks, int k1, double Nd, int tid,
                                             T &pe, T &pmx, T &pmy, T &pmz)
{
    const int n_therm = in.n_therm, trace_sweeps = in.trace_sweeps, wave = tid >> 6, wl = tid & 63;
    const double J = in.J;
    const bool meas = ks >= n_therm || ks < trace_sweeps || ks == k1 - 1;
    if (meas) {
        pe = row_sum(pe);
        pmx = row_sum(pmx);
        pmy = row_sum(pmy);
        pmz = row_sum(pmz);
        if ((wl & 15) == 0) {
            T *slot = g.red + 4 * (tid >> 4);
            slot[0] = pe;
            slot[1] = pmx;
            slot[2] = pmy;
            slot[3] = pmz;
        }
    }
    __syncthreads();
    if (meas && g.active && wave == 0) {
        T se = T(0), sx = T(0), sy = T(0), sz = T(0);
        if (wl < 4 * W) {
            se = g.red[4 * wl + 0];
            sx = g.red[4 * wl + 1];
            sy = g.red[4 * wl + 2];
            sz = g.red[4 * wl + 3];
        }
        se = wave_sum(se);
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        sz = wave_sum(sz);
        if (wl == 0) {
            const double e = -J * (double)se / Nd;
            const double mx = (double)sx / Nd, my = (double)sy / Nd, mz = (double)sz / Nd;
            if (ks >= n_therm) {
                const double m = sqrt(mx * mx + my * my + mz * mz);
                g.shacc[0] += e;
                g.shacc[1] += e * e;
                g.shacc[2] += m;
                g.shacc[3] += m * m;
                g.shacc[4] += (m * m) * (m * m);
            }
            if (ks < trace_sweeps) {
                double *tr = in.trace + ((size_t)g.path * trace_sweeps + ks) * 4;
                tr[0] = e;
                tr[1] = mx;
                tr[2] = my;
                tr[3] = mz;
            }
            if (ks == k1 - 1) {
                g.shacc[5] = e;
                g.shacc[6] = mx;
                g.shacc[7] = my;
                g.shacc[8] = mz;
            }
        }
    }
}

// Sweeps [k0, k1) of one path (the whole workgroup) through the ring. Waves of even index run
// stage 0, odd ones stage 1.
template <typename T, int LC, int B>
__device__ __forceinline__ void path_sweeps_ring(const GroupCtx<T> &g, const InstDev &in, int k0, int k1, bool fresh,
                                                 T *ring)
{
    constexpr int L = LC, HL = L / 2, PLANE = L * L / 2, W = B / 64, SL = B / 2, K = (PLANE + SL - 1) / SL;
    static_assert(W % 2 == 0 && (PLANE % RingRegs<T, LC, B>::E) == 0 && L > RING, "ring shape");
    constexpr bool FP32 = std::is_same<T, float>::value;
    const double Nd = (double)L * L * L;
    const int renorm_every = in.renorm_every;
    Coef<T> cf;
    cf.beta = (T)in.beta;
    cf.J = (T)in.J;
    cf.q = (float)(in.beta * in.J * 1.4426950408889634);  // beta J log2(e)
    const int tid = g.lane, wave = tid >> 6, wl = tid & 63;
    const bool odd_wave = (wave & 1) != 0;
    unsigned long long nacc = 0;
    T *const gsp = g.sp;

    if (g.active && fresh) init_path<T, B>(gsp, nullptr, nullptr, L, tid, g.path, g.key0, g.key1, g.ctr3, in.init);
    // this lane's sites (the same in every plane and for both stages)
    RingSite q[K];
    {
        int lane = tid;
        asm volatile("" : "+v"(lane));  // not hoisted out of a persistent kernel's item loop
        const int rank = (lane >> 6) >> 1, l64 = lane & 63;
#pragma unroll
        for (int t = 0; t < (ring_compact<LC, B>() ? 1 : K); ++t) {
            const int sidx = rank * 64 + l64 + SL * t;
            const int jx = sidx % HL, y = sidx / HL;
            q[t].s = sidx;
            q[t].y = y;
            q[t].idb = 2 * jx + L * y;
            q[t].ypar = y & 1;
            q[t].xm0 = (jx == 0) ? HL - 1 : -1;
            q[t].xp1 = (jx == HL - 1) ? -(HL - 1) : 1;
            q[t].ym = (y == 0) ? (L - 1) * HL : -HL;
            q[t].yp = (y == L - 1) ? -(L - 1) * HL : HL;
        }
    }
    __syncthreads();
    for (int ks = k0; ks < k1; ++ks) {
        const bool rn = FP32 && renorm_every > 0 && ks > 0 && ks % renorm_every == 0;
        // the pass starts with colour 0 of plane 0 and colour 1 of planes -1, 0, 1
        if (g.active) {
            RingRegs<T, LC, B> r;
            ring_load<T, LC, B>(r, gsp, 0, 0, true, 1, L - 1, true, tid);
            ring_store<T, LC, B>(r, ring, 0, 0, true, rn, 1, RING - 1, true, rn, tid);
            ring_load<T, LC, B>(r, gsp, 1, 0, true, 1, 1, true, tid);
            ring_store<T, LC, B>(r, ring, 1, 0, true, rn, 1, 1, true, rn, tid);
        }
        __syncthreads();
        T pe = T(0), pmx = T(0), pmy = T(0), pmz = T(0);
#pragma unroll 1
        for (int tau = 0; tau <= L + 2; ++tau) {
            // next step's half-planes: colour 0 of plane tau + 1 (virtual planes up to L + 1),
            // colour 1 of plane tau + 2 (up to L)
            const bool h0 = tau + 1 <= L + 1, h1 = tau + 2 <= L;
            const int z0 = tau + 1 < L ? tau + 1 : tau + 1 - L, z1 = tau + 2 < L ? tau + 2 : tau + 2 - L;
            RingRegs<T, LC, B> r;
            if (g.active) ring_load<T, LC, B>(r, gsp, 0, z0, h0, 1, z1, h1, tid);
            if (g.active) {
                if (odd_wave) {
                    if (tau >= 3)
                        ring_stage<T, 1, LC, B, K>(g, q, ring, gsp, tau - 2, (uint32_t)ks, cf, rn, pe, pmx, pmy, pmz, nacc);
                } else if (tau < L) {
                    ring_stage<T, 0, LC, B, K>(g, q, ring, gsp, tau, (uint32_t)ks, cf, rn, pe, pmx, pmy, pmz, nacc);
                }
                ring_store<T, LC, B>(r, ring, 0, (tau + 1) % RING, h0, rn && tau + 1 < L, 1, (tau + 2) % RING, h1, rn,
                                     tid);
            }
            __syncthreads();
        }
        ring_measure<T, W>(g, in, ks, k1, Nd, tid, pe, pmx, pmy, pmz);
        // (the next pass's first stores go to the ring, not to the partial slots, which are
        // written again only after L + 3 more barriers)
    }
    if (g.active && wl == 0) atomicAdd((unsigned long long *)&g.shacc[9], nacc);
    __syncthreads();
}

// Sweeps [k0, k1) of one path through the half ring, in two phases per step tau = 0 .. L + 1
// (every lane in each): phase A updates colour 0 of plane tau (tau < L), phase B colour 1 of
// virtual plane tau - 1 (tau >= 2: planes 1 .. L - 1, then 0). Colour 1 of a plane is updated
// only after colour 0 of both its z-neighbours, and colour 0 of a plane reads colour 1 of
// planes tau - 1 .. tau + 1 before any of them is updated (plane 0's colour 1 last of all), so
// the order is that of the sequential half-sweeps. Each step loads colour 0 of plane tau + 1
// (virtual planes up to L + 1) and colour 1 of virtual plane tau + 1 (up to L, plane 0 again
// for the last phase B) into registers and stores them during phase B, into the slot of plane
// tau - 3 and the buffer of plane tau - 1. Phase B reads no buffer: before the first barrier
// each lane copies the spins of its phase-B sites from the buffer of plane tau - 1 into
// registers. So a colour-1 plane is fetched from device memory once per pass (with the
// colour-0 plane below it, whose z-neighbour reads of it hit the L2), not again for its update.
template <typename T, int LC, int B>
__device__ __forceinline__ void path_sweeps_hring(const GroupCtx<T> &g, const InstDev &in, int k0, int k1,
                                                  bool fresh, T *ring)
{
    constexpr int L = LC, HL = L / 2, PLANE = L * L / 2, HALF = L * PLANE, SLOT = 3 * PLANE, W = B / 64,
                  K = (PLANE + B - 1) / B;
    static_assert((PLANE % RingRegs<T, LC, B>::E) == 0 && L > RING, "ring shape");
    constexpr bool FP32 = std::is_same<T, float>::value;
    const double Nd = (double)L * L * L;
    const int renorm_every = in.renorm_every;
    Coef<T> cf;
    cf.beta = (T)in.beta;
    cf.J = (T)in.J;
    cf.q = (float)(in.beta * in.J * 1.4426950408889634);  // beta J log2(e)
    const int tid = g.lane, wl = tid & 63;
    unsigned long long nacc = 0;
    T *const gsp = g.sp;

    if (g.active && fresh) init_path<T, B>(gsp, nullptr, nullptr, L, tid, g.path, g.key0, g.key1, g.ctr3, in.init);
    // this lane's sites of a plane's colour (the same in every plane and for both colours)
    RingSite q[K];
    {
        int lane = tid;
        asm volatile("" : "+v"(lane));  // not hoisted out of a persistent kernel's item loop
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const int sidx = lane + B * t;
            const int jx = sidx % HL, y = sidx / HL;
            q[t].s = sidx;
            q[t].y = y;
            q[t].idb = 2 * jx + L * y;
            q[t].ypar = y & 1;
            q[t].xm0 = (jx == 0) ? HL - 1 : -1;
            q[t].xp1 = (jx == HL - 1) ? -(HL - 1) : 1;
            q[t].ym = (y == 0) ? (L - 1) * HL : -HL;
            q[t].yp = (y == L - 1) ? -(L - 1) * HL : HL;
        }
    }
    __syncthreads();
    for (int ks = k0; ks < k1; ++ks) {
        const bool rn = FP32 && renorm_every > 0 && ks > 0 && ks % renorm_every == 0;
        // colour 1 stays in device memory: normalised in place before a renormalisation pass
        if constexpr (FP32) if (rn && g.active) {
            T *const c1 = gsp + 3 * HALF;
            for (int t = tid; t < HALF; t += B) {
                const T x = c1[t], y = c1[HALF + t], z = c1[2 * HALF + t];
                const float rr = __builtin_amdgcn_rsqf(fmaf(z, z, fmaf(y, y, x * x)));
                c1[t] = x * rr;
                c1[HALF + t] = y * rr;
                c1[2 * HALF + t] = z * rr;
            }
        }
        if (rn) __syncthreads();  // (uniform) normalised before planes 0 and L - 1 are read below
        // the pass starts with colour 0 of plane 0 in slot 0, colour 1 of plane 0 in buffer 0 and
        // colour 1 of plane L - 1 (below plane 0) in buffer 1
        if (g.active) {
            RingRegs<T, LC, B> r;
            ring_load<T, LC, B>(r, gsp, 0, 0, true, 1, 0, true, tid);
            ring_store<T, LC, B, true>(r, ring, 0, 0, true, rn, 1, 0, true, false, tid);
            ring_load<T, LC, B>(r, gsp, 0, 0, false, 1, L - 1, true, tid);
            ring_store<T, LC, B, true>(r, ring, 0, 0, false, false, 1, 1, true, false, tid);
        }
        __syncthreads();
        T pe = T(0), pmx = T(0), pmy = T(0), pmz = T(0);
#pragma unroll 1
        for (int tau = 0; tau <= L + 1; ++tau) {
            const bool h0 = tau + 1 <= L + 1, h1 = tau + 1 <= L;
            const int z0 = tau + 1 < L ? tau + 1 : tau + 1 - L, z1 = tau + 1 < L ? tau + 1 : 0;
            RingRegs<T, LC, B> r;
            if (g.active) ring_load<T, LC, B>(r, gsp, 0, z0, h0, 1, z1, h1, tid);
            // phase B's own spins (colour 1 of plane tau - 1, in the buffer the step replaces)
            T own1[K][3];
            if (g.active && tau >= 2) {
                const T *const b = ring + HR_SLOTS * SLOT + ((tau - 1) & 1) * SLOT;
#pragma unroll
                for (int t = 0; t < K; ++t) {
                    const int h = q[t].s < PLANE ? q[t].s : 0;  // (sites past the plane are not updated)
                    own1[t][0] = b[h];
                    own1[t][1] = b[PLANE + h];
                    own1[t][2] = b[2 * PLANE + h];
                }
            }
            if (g.active && tau < L)
                hring_stage<T, 0, LC, B, K>(g, q, own1, ring, gsp, tau, (uint32_t)ks, cf, rn, pe, pmx, pmy, pmz, nacc);
            __syncthreads();
            if (g.active) {
                if (tau >= 2)
                    hring_stage<T, 1, LC, B, K>(g, q, own1, ring, gsp, tau - 1, (uint32_t)ks, cf, rn, pe, pmx, pmy, pmz,
                                                nacc);
                ring_store<T, LC, B, true>(r, ring, 0, (tau + 1) % HR_SLOTS, h0, rn && tau + 1 < L, 1, (tau + 1) & 1,
                                           h1, false, tid);
            }
            __syncthreads();
        }
        ring_measure<T, W>(g, in, ks, k1, Nd, tid, pe, pmx, pmy, pmz);
    }
    if (g.active && wl == 0) atomicAdd((unsigned long long *)&g.shacc[9], nacc);
    __syncthreads();
}

// ------------------------------------------------------------------ two-sweep plane ring
// Stage codes of a phase of the two-sweep ring; R2_COPY: copy registers of colour 0 of a
// reloaded virtual plane (L .. L + 3) into its slot.
enum { R2_S0 = 0, R2_S1 = 1, R2_S2 = 2, R2_S3 = 3, R2_COPY = 4, R2_NONE = 5 };

constexpr int ring2_gcd(int a, int b) { return b == 0 ? a : ring2_gcd(b, a % b); }

template <typename T, int LC, int B>
struct Ring2Shape {
    static constexpr int HL = LC / 2, PLANE = LC * LC / 2, HALF = LC * PLANE;
    // a lane's sites in any plane are congruent modulo G; COMPACT: G is whole rows (DY of them),
    // so they share their x position and one site's geometry serves all
    static constexpr int G = ring2_gcd(B, PLANE), DY = G / HL;
    static constexpr bool COMPACT = G % HL == 0;
    static constexpr int RMAX = (2 * PLANE + B - 1) / B;  // rounds of a phase with two stages
    static constexpr int KS = (PLANE + B - 1) / B;        // rounds of the first stage of a phase
    // a colour-plane component moves between device memory and LDS in groups of E consecutive
    // sites, as narrow as lets every group have a lane (few registers held per lane)
    static constexpr int EMAX = 16 / (int)sizeof(T);
    static constexpr int E = PLANE <= B ? 1 : (PLANE <= 2 * B || EMAX == 2) ? 2 : 4;
    static constexpr int NQ = PLANE / E, RQ = (NQ + B - 1) / B;
};

template <typename T, int E> struct R2Vec { using type = T; };
template <> struct R2Vec<float, 2> { using type = float2; };
template <> struct R2Vec<float, 4> { using type = float4; };
template <> struct R2Vec<double, 2> { using type = double2; };

// Geometry of the lane's site r = lane mod G of a plane (row yr, x-pair 2 jx = idx); its
// site of round i in region a is r + G m with m = q + (B / G) i - (plane / G) a (compact
// shapes; otherwise (lane + B i) mod plane, kept per round with its row in s, y).
template <int RMAX>
struct Ring2Lane {
    int r, yr, q, idx, xm0, xp1;
    int s[RMAX], y[RMAX];
};

template <int... I, typename F>
__device__ __forceinline__ void unroll_each(std::integer_sequence<int, I...>, F &&f)
{
    (f(std::integral_constant<int, I>{}), ...);
}

// Colour c of virtual plane v (v >= -1) in the two-sweep ring's LDS.
template <int PLANE, typename T>
__device__ __forceinline__ T *ring2_slot(T *ring, int c, int v)
{
    return c ? ring + 3 * PLANE * (R2_SLOTS0 + (v + R2_SLOTS1) % R2_SLOTS1) : ring + 3 * PLANE * ((v + R2_SLOTS0) % R2_SLOTS0);
}

// One Metropolis attempt of stage ST (colour ST & 1) of the two-sweep ring at the lane's site s
// (row y) of virtual plane v, sweep k. own, oth, othm, othp: the LDS slots of the stage's
// colour in plane v and of the other colour in planes v, v - 1, v + 1 (the caller's per-step
// slot pointers); own_r: the spin when stage 0 or 3 takes it from registers; zm_r: stage 3's
// neighbour below (registers; its othm is not read); wglob: stage 0 / 1 also writes accepted
// moves to device memory.
template <typename T, int ST, int LC, int B, typename Lane>
__device__ __forceinline__ void ring2_site(const GroupCtx<T> &g, const Lane &ln, int s, int y, int v, uint32_t k,
                                           T *own, const T *oth, const T *othm, const T *othp, T *gsp,
                                           const T (&own_r)[3], const T (&zm_r)[3], bool wglob,
                                           const Coef<T> &cf, T &pe, T &pmx, T &pmy, T &pmz,
                                           unsigned long long &nacc)
{
    using S = Ring2Shape<T, LC, B>;
    constexpr int L = LC, HL = S::HL, PLANE = S::PLANE, HALF = S::HALF, C = ST & 1;
    int idx, xm0, xp1;
    if constexpr (S::COMPACT) {
        idx = ln.idx;
        xm0 = ln.xm0;
        xp1 = ln.xp1;
    } else {
        const int jx = s - HL * y;
        idx = 2 * jx;
        xm0 = (jx == 0) ? HL - 1 : -1;
        xp1 = (jx == HL - 1) ? -(HL - 1) : 1;
    }
    const int zp = v < L ? v : v - L;  // (0 <= v < 2L)
    const int p = (y + zp + C) & 1;
    Site st;
    st.h = s;
    st.id = idx + p + L * y + L * L * zp;
    // in-plane neighbours (plane-local indices); the z-neighbours share s
    st.nb[0] = s + (p ? 0 : xm0);
    st.nb[1] = s + (p ? xp1 : 0);
    st.nb[2] = s + ((y == 0) ? (L - 1) * HL : -HL);
    st.nb[3] = s + ((y == L - 1) ? -(L - 1) * HL : HL);
    st.nb[4] = st.nb[5] = s;
    // this colour in device memory, indexed from each component's start: zb the first site of
    // plane zp
    T *const gown = gsp + C * 3 * HALF;
    const int zb = zp * PLANE;
    update_site_f<T, false>(
        g, C != 0, st, k, cf, pe, pmx, pmy, pmz, nacc,
        [&](int c) { return (ST == R2_S0 || ST == R2_S3) ? own_r[c] : own[c * PLANE + s]; },
        [&](int c, int n) -> T {
            if (n < 4) return oth[c * PLANE + st.nb[n]];
            if (n == 4) {
                if constexpr (ST == R2_S3) return zm_r[c];
                else return othm[c * PLANE + s];
            }
            return othp[c * PLANE + s];
        },
        [&](bool acc, T nx, T ny, T nz, T sx, T sy, T sz) {
            if constexpr (ST == R2_S0) {
                own[s] = acc ? nx : sx;
                own[PLANE + s] = acc ? ny : sy;
                own[2 * PLANE + s] = acc ? nz : sz;
            } else if constexpr (ST == R2_S3) {
                spin_at<true>(gown, zb + s) = acc ? nx : sx;
                spin_at<true>(gown + HALF, zb + s) = acc ? ny : sy;
                spin_at<true>(gown + 2 * HALF, zb + s) = acc ? nz : sz;
            } else {
                if (acc) {
                    own[s] = nx;
                    own[PLANE + s] = ny;
                    own[2 * PLANE + s] = nz;
                }
            }
            if constexpr (ST == R2_S0 || ST == R2_S1) {
                if (wglob && acc) {
                    spin_at<true>(gown, zb + s) = nx;
                    spin_at<true>(gown + HALF, zb + s) = ny;
                    spin_at<true>(gown + 2 * HALF, zb + s) = nz;
                }
            }
        });
}

// Sweeps [k0, k1) of one path (the whole workgroup) through the two-sweep ring: passes of two
// sweeps, one-sweep passes where two cannot be taken (see the placement notes above).
template <typename T, int LC, int B>
__device__ __forceinline__ void path_sweeps_ring2(const GroupCtx<T> &g, const InstDev &in, int k0, int k1, bool fresh,
                                                  T *ring)
{
    using S = Ring2Shape<T, LC, B>;
    using V = typename R2Vec<T, S::E>::type;
    constexpr int L = LC, HL = S::HL, PLANE = S::PLANE, HALF = S::HALF, W = B / 64;
    constexpr int G = S::G, RMAX = S::RMAX, KS = S::KS, E = S::E, NQ = S::NQ, RQ = S::RQ;
    static_assert(B % 64 == 0 && PLANE % 64 == 0 && PLANE % E == 0 && L > RING, "two-sweep ring shape");
    constexpr uint32_t CB = HALF * sizeof(T);  // bytes between components
    constexpr bool FP32 = std::is_same<T, float>::value;
    const double Nd = (double)L * L * L;
    const int renorm_every = in.renorm_every;
    Coef<T> cf;
    cf.beta = (T)in.beta;
    cf.J = (T)in.J;
    cf.q = (float)(in.beta * in.J * 1.4426950408889634);  // beta J log2(e)
    const int tid = g.lane, wl = tid & 63;
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);  // the wave's first lane
    unsigned long long nacc = 0;
    T *const gsp = g.sp;

    if (g.active && fresh) init_path<T, B>(gsp, nullptr, nullptr, L, tid, g.path, g.key0, g.key1, g.ctr3, in.init);
    Ring2Lane<RMAX> ln;
    {
        int lane = tid;
        asm volatile("" : "+v"(lane));  // not hoisted out of a persistent kernel's item loop
        if constexpr (S::COMPACT) {
            ln.r = lane % G;
            ln.q = lane / G;
            const int jx = ln.r % HL;
            ln.yr = ln.r / HL;
            ln.idx = 2 * jx;
            ln.xm0 = (jx == 0) ? HL - 1 : -1;
            ln.xp1 = (jx == HL - 1) ? -(HL - 1) : 1;
        } else {
#pragma unroll
            for (int i = 0; i < RMAX; ++i) {
                const int u = lane + B * i;
                ln.s[i] = u - (u / PLANE) * PLANE;
                ln.y[i] = ln.s[i] / HL;
            }
        }
    }
    // the lane's site of round i in region a (a = (lane + B i) / plane)
    auto site_of = [&](int i, int a, int &s, int &y) {
        if constexpr (S::COMPACT) {
            const int m = ln.q + (B / G) * i - (PLANE / G) * a;
            s = ln.r + G * m;
            y = ln.yr + S::DY * m;
        } else {
            s = ln.s[i];
            y = ln.y[i];
        }
    };
    __syncthreads();
    // colour c of plane zp from device memory into registers, 16-byte groups j = tid + B jj
    auto load_plane = [&](V (&r)[RQ][3], int c, int zp) {
#pragma unroll
        for (int jj = 0; jj < RQ; ++jj) {
            const int j = tid + B * jj;
            if ((NQ % B) == 0 || j < NQ) {
                const uint32_t off = (uint32_t)(c * 3 * HALF + zp * PLANE + E * j) * (uint32_t)sizeof(T);
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) r[jj][cc] = ld16<V>(gsp, off + cc * CB);
            }
        }
    };
    auto store_half = [&](const V (&r)[RQ][3], T *half) {
#pragma unroll
        for (int jj = 0; jj < RQ; ++jj) {
            const int j = tid + B * jj;
            if ((NQ % B) == 0 || j < NQ) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) *reinterpret_cast<V *>(half + cc * PLANE + E * j) = r[jj][cc];
            }
        }
    };
    // colour 0 of plane zp at the lane's sites of a phase's first stage (rounds i < KS)
    auto load_own0 = [&](T (&o)[KS][3], int zp) {
#pragma unroll
        for (int i = 0; i < KS; ++i) {
            const int s = tid + B * i;
            if ((PLANE % B) == 0 || s < PLANE) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) o[i][cc] = spin_at<true>(gsp + cc * HALF, zp * PLANE + s);
            }
        }
    };

    for (int ks = k0; ks < k1;) {
        const bool rn = FP32 && renorm_every > 0 && ks > 0 && ks % renorm_every == 0;
        const bool two = ks + 1 < k1 && !(FP32 && renorm_every > 0 && (ks + 1) % renorm_every == 0);
        if constexpr (FP32) {
            if (rn && g.active) renorm_path<B>(gsp, nullptr, nullptr, L, tid);
            if (rn) __syncthreads();  // (uniform) normalised before any plane is read below
        }
        // colour 1 of planes -1, 0 and 1 into their slots, colour 0 of plane 0 into registers
        T own0[KS][3];
        if (g.active) {
            V r[RQ][3];
            load_plane(r, 1, L - 1);
            store_half(r, ring2_slot<PLANE>(ring, 1, -1));
            load_plane(r, 1, 0);
            store_half(r, ring2_slot<PLANE>(ring, 1, 0));
            load_plane(r, 1, 1);
            store_half(r, ring2_slot<PLANE>(ring, 1, 1));
            load_own0(own0, 0);
        }
        __syncthreads();
        const int nsteps = two ? L + 7 : L + 2, c1_last = two ? L + 2 : L, c0_last = two ? L + 3 : L + 1;
        T pA[4] = {T(0), T(0), T(0), T(0)}, pB[4] = {T(0), T(0), T(0), T(0)};  // partials of sweeps ks, ks + 1
        T own3[RMAX][3], zm3[RMAX][3];  // stage 3's own spins and neighbours below
        int i0 = 0, i1 = 0;  // tau mod R2_SLOTS0, tau mod R2_SLOTS1
#pragma unroll 1
        for (int tau = 0; tau < nsteps; ++tau) {
            // the step's slots, from the running indices (no division per update): colour 0 of
            // plane tau - d (d = 0 .. 4), colour 1 of plane tau - d (d = -1 .. 4)
            auto c0s = [&](int d) { int j = i0 - d; j += j < 0 ? R2_SLOTS0 : 0; return ring + 3 * PLANE * j; };
            auto c1s = [&](int d) {
                int j = i1 - d;
                j += j < 0 ? R2_SLOTS1 : 0;
                j -= j >= R2_SLOTS1 ? R2_SLOTS1 : 0;
                return ring + 3 * PLANE * (R2_SLOTS0 + j);
            };
            T *const c0_0 = c0s(0), *const c0_1 = c0s(1), *const c0_2 = c0s(2), *const c0_3 = c0s(3), *const c0_4 = c0s(4);
            T *const c1_p1 = c1s(-1), *const c1_0 = c1s(0), *const c1_1 = c1s(1), *const c1_2 = c1s(2),
                     *const c1_3 = c1s(3), *const c1_4 = c1s(4);
            // colour 1 of virtual plane tau + 2 (stored in phase 2) and colour 0 of plane tau + 1
            // (the next step's first stage's own spins) into registers
            const bool h1 = tau + 2 <= c1_last, h0 = tau + 1 <= c0_last;
            const int z1 = tau + 2 < L ? tau + 2 : tau + 2 - L, z0 = tau + 1 < L ? tau + 1 : tau + 1 - L;
            V r1[RQ][3];
            T own0n[KS][3];
            if (g.active && h1) load_plane(r1, 1, z1);
            if (g.active && h0) load_own0(own0n, z0);
            // phase 1 (colour 0): stage 0 or the copy of a reloaded plane, then stage 2
            const int f1 = tau < L ? R2_S0 : (tau <= c0_last ? R2_COPY : R2_NONE);
            const bool s2 = two && tau >= 5 && tau < L + 5, s1 = tau >= 2 && tau < L + 2,
                       s3 = two && tau >= 7 && tau < L + 7;
            const int n1 = (f1 != R2_NONE ? 1 : 0) + (s2 ? 1 : 0), first1 = f1 != R2_NONE ? f1 : R2_S2;
            if (g.active) {
                unroll_each(std::make_integer_sequence<int, RMAX>{}, [&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    const int a = (wbase + B * i) / PLANE;  // region (wave-uniform)
                    if (a < n1) {
                        int s, y;
                        site_of(i, a, s, y);
                        const int stg = a == 0 ? first1 : R2_S2;
                        if constexpr (i < KS) {
                            if (stg == R2_S0) {
                                ring2_site<T, R2_S0, LC, B>(g, ln, s, y, tau, (uint32_t)ks, c0_0, c1_0, c1_1, c1_p1, gsp,
                                                            own0[i], own0[i], !two, cf, pA[0], pA[1], pA[2], pA[3], nacc);
                                return;
                            }
                            if (stg == R2_COPY) {
                                T *const o = c0_0;
                                o[s] = own0[i][0];
                                o[PLANE + s] = own0[i][1];
                                o[2 * PLANE + s] = own0[i][2];
                                return;
                            }
                        }
                        ring2_site<T, R2_S2, LC, B>(g, ln, s, y, tau - 3, (uint32_t)(ks + 1), c0_3, c1_3, c1_4, c1_2,
                                                    gsp, own0[0], own0[0], false, cf, pB[0], pB[1], pB[2], pB[3], nacc);
                    }
                });
                if (s3) {
                    // stage 3's own spins (colour 1 of plane tau - 4), before phase 2 replaces them
                    const int a3 = s1 ? 1 : 0;
                    const T *const src = c1_4;
                    unroll_each(std::make_integer_sequence<int, RMAX>{}, [&](auto ic) {
                        constexpr int i = decltype(ic)::value;
                        if ((wbase + B * i) / PLANE == a3) {
                            int s, y;
                            site_of(i, a3, s, y);
                            own3[i][0] = src[s];
                            own3[i][1] = src[PLANE + s];
                            own3[i][2] = src[2 * PLANE + s];
                        }
                    });
                }
                if (two && tau >= 4 && tau <= L + 5) {
                    // colour 0 of plane tau - 4 back to device memory (final for this pass)
                    const int v = tau - 4, zp = v < L ? v : v - L;
                    const T *const src = c0_4;
#pragma unroll
                    for (int jj = 0; jj < RQ; ++jj) {
                        const int j = tid + B * jj;
                        if ((NQ % B) == 0 || j < NQ) {
#pragma unroll
                            for (int cc = 0; cc < 3; ++cc)
                                *reinterpret_cast<V *>(gsp + cc * HALF + zp * PLANE + E * j) =
                                    *reinterpret_cast<const V *>(src + cc * PLANE + E * j);
                        }
                    }
                }
            }
            __syncthreads();
            // phase 2 (colour 1): stage 1, then stage 3
            if (g.active) {
                const int n2 = (s1 ? 1 : 0) + (s3 ? 1 : 0), first2 = s1 ? R2_S1 : R2_S3;
                unroll_each(std::make_integer_sequence<int, RMAX>{}, [&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    const int a = (wbase + B * i) / PLANE;
                    if (a < n2) {
                        int s, y;
                        site_of(i, a, s, y);
                        if ((a == 0 ? first2 : R2_S3) == R2_S1)
                            ring2_site<T, R2_S1, LC, B>(g, ln, s, y, tau - 1, (uint32_t)ks, c1_1, c0_1, c0_2, c0_0, gsp,
                                                        own3[i], zm3[i], !two || tau - 1 <= 2, cf, pA[0], pA[1], pA[2],
                                                        pA[3], nacc);
                        else
                            ring2_site<T, R2_S3, LC, B>(g, ln, s, y, tau - 4, (uint32_t)(ks + 1), c1_4, c0_4, c0_4, c0_3,
                                                        gsp, own3[i], zm3[i], false, cf, pB[0], pB[1], pB[2], pB[3],
                                                        nacc);
                    }
                });
                if (h1) store_half(r1, c1_4);  // (plane tau + 2 takes the slot of tau - 4)
                // the next step's stage 3 neighbours below: colour 0 of plane tau - 4, in its slot
                // until phase 1 of the next step (this lane's stage-3 updates above have read zm3)
                if (two && tau + 1 >= 7 && tau + 1 < L + 7) {
                    const int a3 = (tau + 1 >= 2 && tau + 1 < L + 2) ? 1 : 0;
                    const T *const src = c0_4;
                    unroll_each(std::make_integer_sequence<int, RMAX>{}, [&](auto ic) {
                        constexpr int i = decltype(ic)::value;
                        if ((wbase + B * i) / PLANE == a3) {
                            int s, y;
                            site_of(i, a3, s, y);
                            zm3[i][0] = src[s];
                            zm3[i][1] = src[PLANE + s];
                            zm3[i][2] = src[2 * PLANE + s];
                        }
                    });
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < KS; ++i) {
                own0[i][0] = own0n[i][0];
                own0[i][1] = own0n[i][1];
                own0[i][2] = own0n[i][2];
            }
            i0 = i0 == R2_SLOTS0 - 1 ? 0 : i0 + 1;
            i1 = i1 == R2_SLOTS1 - 1 ? 0 : i1 + 1;
        }
        ring_measure<T, W>(g, in, ks, k1, Nd, tid, pA[0], pA[1], pA[2], pA[3]);
        if (two) {
            __syncthreads();  // (wave 0 has read the partials of sweep ks)
            ring_measure<T, W>(g, in, ks + 1, k1, Nd, tid, pB[0], pB[1], pB[2], pB[3]);
        }
        ks += two ? 2 : 1;
    }
    if (g.active && wl == 0) atomicAdd((unsigned long long *)&g.shacc[9], nacc);
    __syncthreads();
}

template <typename T, int LC, int B, int PL>
__device__ __forceinline__ void wg_run_ring(const InstDev &in, int path, int k0, int k1, bool fresh, char *smem, T *gsp)
{
    GroupCtx<T> g;
    g.L = in.L;
    g.lane = threadIdx.x;
    g.path = (uint32_t)__builtin_amdgcn_readfirstlane(path);
    g.key0 = in.key0;
    g.key1 = in.key1;
    g.ctr3 = in.ctr3;
    g.active = path < in.n_paths;
    T *ring = reinterpret_cast<T *>(smem);
    char *p = smem + ring_lds_bytes<T>(LC, B, PL) - 128 - (size_t)(B / 16) * 4 * sizeof(T);
    g.shacc = reinterpret_cast<double *>(p);
    g.red = reinterpret_cast<T *>(p + 128);
    g.sp = gsp;
    g.sp1 = nullptr;
    g.sp0z = nullptr;
    load_acc(g.shacc, in.acc + g.path, fresh, g.lane, g.active);
    if constexpr (PL == PL_HRING) path_sweeps_hring<T, LC, B>(g, in, k0, k1, fresh, ring);
    else if constexpr (PL == PL_RING2) path_sweeps_ring2<T, LC, B>(g, in, k0, k1, fresh, ring);
    else path_sweeps_ring<T, LC, B>(g, in, k0, k1, fresh, ring);
    store_acc(g.shacc, in.acc + g.path, g.lane, g.active);
}

// Sets up the group views of one workgroup and runs sweeps [k0, k1) for paths
// path0 + group. gbase: device memory of path path0's spins (group g at gbase + g * 3 L^3):
// the instance's resident array (resident = true: LDS spins are loaded from and stored back
// to it) or a batch slot. The caller passes the base explicitly: a select between the two
// crashes the ROCm 7.2 optimizer (SimplifyCFG). PL: a Place; with PL_SPLIT colour 1 is swept
// in place in device memory and only colour 0 is copied to and from LDS (PL_SPLIT_XY: only
// colour 0's x and y).
template <typename T, int LC, int G, int B, int MAP, int PL>
__device__ __forceinline__ void wg_run_groups(const InstDev &in, int path0, int k0, int k1, bool fresh, char *smem,
                                              T *gbase, bool resident)
{
    constexpr bool IN_LDS = PL != PL_MEM;
    constexpr int P = B / G;
    const int L = LC ? LC : in.L;
    const size_t NS = 3 * (size_t)L * L * L;  // spin words per path
    const int group = threadIdx.x / G;
    GroupCtx<T> g;
    g.L = in.L;
    g.lane = threadIdx.x % G;
    // wave-uniform by construction (G is a multiple of 64): keep in scalar registers
    g.path = (uint32_t)__builtin_amdgcn_readfirstlane(path0 + group);
    g.key0 = in.key0;
    g.key1 = in.key1;
    g.ctr3 = in.ctr3;
    g.active = (int)g.path < in.n_paths;
    char *p = smem;
    T *lds_spins = reinterpret_cast<T *>(p);
    // spin words of a path held in LDS (colour 0's x and y come first in the path's array)
    const size_t NL = PL == PL_LDS ? NS : PL == PL_SPLIT ? NS / 2 : PL == PL_SPLIT_XY ? NS / 3 : 0;
    p += P * NL * sizeof(T);
    g.shacc = reinterpret_cast<double *>(p) + 16 * group;
    p += P * 128;
    g.red = reinterpret_cast<T *>(p) + 16 * (group * (G / 64));
    T *gsp = gbase + (size_t)group * NS;
    g.sp = IN_LDS ? lds_spins + (size_t)group * NL : gsp;
    g.sp1 = PL == PL_LDS ? g.sp + NS / 2 : gsp + NS / 2;
    g.sp0z = gsp + NS / 3;

    load_acc(g.shacc, in.acc + g.path, fresh, g.lane, g.active);
    if (IN_LDS && !fresh && g.active) copy_spins<G>(g.sp, gsp, (int)NL, g.lane);
    // (path_sweeps begins with a barrier)
    path_sweeps<T, LC, G, MAP, PL>(g, in, k0, k1, fresh);
    if (IN_LDS && resident && g.active) copy_spins<G>(gsp, g.sp, (int)NL, g.lane);
    store_acc(g.shacc, in.acc + g.path, g.lane, g.active);
}

template <typename T, int LC, int G, int B, int MAP, int PL>
__device__ __forceinline__ void wg_run(const InstDev &in, int path0, int k0, int k1, bool fresh, char *smem, T *gbase,
                                       bool resident)
{
    if constexpr (PL == PL_RING || PL == PL_HRING || PL == PL_RING2) {
        static_assert(G == B, "one path per workgroup");
        wg_run_ring<T, LC, B, PL>(in, path0, k0, k1, fresh, smem, gbase);
    } else {
        wg_run_groups<T, LC, G, B, MAP, PL>(in, path0, k0, k1, fresh, smem, gbase, resident);
    }
}

// Waves per SIMD a kernel variant aims for (the compiler sizes its registers to fit): as
// many workgroups as the 160 KiB of LDS per CU holds, 4 SIMDs per CU, at most 8 waves per
// SIMD (4 in FP64); 4 (FP64: 2) for spins in device memory.
template <typename T>
constexpr int target_waves(int L, int B, int G, int pl)
{
    const int fp64 = sizeof(T) == 8;  // FP64 values take register pairs
    if (pl == PL_MEM || L == 0) return fp64 ? 2 : 4;
    const int wgs = (int)((size_t)160 * 1024 / lds_layout_bytes<T>(L, B, G, pl));
    // (the plane ring keeps a whole update's worth of geometry and in-flight planes per lane)
    const int w = wgs * (B / 64) / 4,
              cap = (pl == PL_RING || pl == PL_HRING || pl == PL_RING2) ? (fp64 ? 2 : 4) : (fp64 ? 4 : 8);
    return w < 1 ? 1 : (w > cap ? cap : w);
}

template <typename T, int LC, int G, int B, int MAP, int PL>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(target_waves<T>(LC, B, G, PL))))
void k_resident(InstDev in, int k0, int k1, int fresh)
{
    extern __shared__ __align__(16) char smem[];
    const int L = LC ? LC : in.L;
    const int path0 = blockIdx.x * (B / G);
    wg_run<T, LC, G, B, MAP, PL>(in, path0, k0, k1, fresh != 0, smem,
                                     reinterpret_cast<T *>(in.spins) + (size_t)path0 * 3 * L * L * L, true);
}

template <typename T, int LC, int G, int B, int MAP, int PL>
hipError_t launch_resident(const InstDev &in, int k0, int k1, int fresh, hipStream_t s)
{
    const int L = LC ? LC : in.L;
    const size_t lds = lds_layout_bytes<T>(L, B, G, PL);
    auto kern = k_resident<T, LC, G, B, MAP, PL>;
    const int grid = (in.n_paths + (B / G) - 1) / (B / G);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(B), lds, s, in, k0, k1, fresh);
    return hipGetLastError();
}

// ------------------------------------------------------------------ z-pipelined window
// For lattices whose spins do not fit in LDS: the path's spins stay in device memory and the
// workgroup (one path) runs D sweeps per pass over them, holding a sliding window of
// z-planes (both colours, three components) in LDS. Stage j = 2d + c of a pass is the
// colour-c half-sweep of sweep ks + d; at step tau it updates every site of colour c in
// virtual plane v = tau - 2j (physical plane v mod L), for v in [j, j + L). Stage j lags
// stage j - 1 by three steps and starts one plane further round the periodic z-ring, so
// each site sees exactly the neighbour values of the sequential half-sweep order (even
// then odd, sweep after sweep), the periodic wrap included; stages that are active in the
// same step touch disjoint data and run together between two barriers. A plane is read from
// device memory into registers four steps before its first use, stored into the window at
// the end of the next step (so the load's latency overlaps a whole step of updates), and
// written back the step after its last use; virtual planes v and v + L are the same physical plane and
// are never in the window together (L > 4D + 4). Device-memory traffic is about
// 24 (1 + (2D + 1)/L) / D bytes per update in FP32 instead of 36.
// Renormalisation boundaries (FP32) always start a pass: the pass normalises every site
// when it first loads its plane, as the resident kernels do at the start of that sweep.
template <typename T>
__host__ __device__ constexpr size_t win_lds_bytes(int L, int B, int D, bool gm = false)
{
    return (gm ? 0 : (size_t)(4 * D + 4) * 3 * (size_t)L * L * sizeof(T)) + 128 + (size_t)D * (B / 64) * 16 * sizeof(T);
}

__device__ __forceinline__ int wrap_mod(int v, int n)
{
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// Waves dealt out over n active stages (1 <= n <= NMAX): wave w serves stage slot w % n as
// the (w / n)-th of its cnt waves. Division by a small runtime n through constant divisors.
template <int M>
__device__ __forceinline__ void deal_by(unsigned w, unsigned nwaves, int &slot, int &rank, int &cnt)
{
    slot = (int)(w % M);
    rank = (int)(w / M);
    cnt = (int)((nwaves - slot + M - 1) / M);
}

template <int NMAX>
__device__ __forceinline__ void deal_waves(int w, int n, int nwaves, int &slot, int &rank, int &cnt)
{
    static_assert(NMAX <= 6, "at most six stages");
    switch (n) {  // wave-uniform: one branch taken
    case 1: slot = 0; rank = w; cnt = nwaves; break;
    case 2: deal_by<2>(w, nwaves, slot, rank, cnt); break;
    case 3: deal_by<3>(w, nwaves, slot, rank, cnt); break;
    case 4: deal_by<4>(w, nwaves, slot, rank, cnt); break;
    case 5: deal_by<5>(w, nwaves, slot, rank, cnt); break;
    default: deal_by<6>(w, nwaves, slot, rank, cnt); break;
    }
}

// Active stages j (3j <= tau < 3j + L) of a pass with nst stages: [lo, hi].
__device__ __forceinline__ void active_stages(int tau, int L, int nst, int &lo, int &hi)
{
    lo = tau >= L ? (tau - L) / 3 + 1 : 0;
    hi = tau / 3 < nst - 1 ? tau / 3 : nst - 1;
}

// One plane (both colours) of a path held by the workgroup's lanes in registers: lane t owns
// the sites t, t + B, ... of the plane's 2 * plane sites (colour-major).
template <typename T, int LC, int B>
struct PlaneRegs {
    static constexpr int PLANE = LC * LC / 2, NPS = (2 * PLANE + B - 1) / B;
    T x[NPS], y[NPS], z[NPS];
};

template <typename T, int LC, int B>
__device__ __forceinline__ void plane_load(PlaneRegs<T, LC, B> &r, const T *gsp, int zp, int tid, bool norm)
{
    constexpr int PLANE = LC * LC / 2, HALF = LC * PLANE, NPS = PlaneRegs<T, LC, B>::NPS;
#pragma unroll
    for (int i = 0; i < NPS; ++i) {
        const int e = tid + B * i;
        if ((2 * PLANE) % B == 0 || e < 2 * PLANE) {
            const int c = e >= PLANE, s = e - c * PLANE;
            const T *q = gsp + c * 3 * HALF + zp * PLANE + s;
            T x = q[0], y = q[HALF], z = q[2 * HALF];
            if constexpr (std::is_same<T, float>::value) {
                if (norm) {
                    const float n = __builtin_amdgcn_rsqf(fmaf(z, z, fmaf(y, y, x * x)));
                    x = x * n;
                    y = y * n;
                    z = z * n;
                }
            }
            r.x[i] = x;
            r.y[i] = y;
            r.z[i] = z;
        }
    }
}

template <typename T, int LC, int B>
__device__ __forceinline__ void plane_to_lds(const PlaneRegs<T, LC, B> &r, T *slot, int tid)
{
    constexpr int PLANE = LC * LC / 2, NPS = PlaneRegs<T, LC, B>::NPS;
#pragma unroll
    for (int i = 0; i < NPS; ++i) {
        const int e = tid + B * i;
        if ((2 * PLANE) % B == 0 || e < 2 * PLANE) {
            const int c = e >= PLANE, s = e - c * PLANE;
            T *q = slot + c * 3 * PLANE + s;
            q[0] = r.x[i];
            q[PLANE] = r.y[i];
            q[2 * PLANE] = r.z[i];
        }
    }
}

template <typename T, int LC, int B>
__device__ __forceinline__ void plane_writeback(const T *slot, T *gsp, int zp, int tid)
{
    constexpr int PLANE = LC * LC / 2, HALF = LC * PLANE;
    for (int e = tid; e < 2 * PLANE; e += B) {
        const int c = e >= PLANE, s = e - c * PLANE;
        const T *q = slot + c * 3 * PLANE + s;
        T *o = gsp + c * 3 * HALF + zp * PLANE + s;
        o[0] = q[0];
        o[HALF] = q[PLANE];
        o[2 * HALF] = q[2 * PLANE];
    }
}

// Adds a wave's register partials of sweep d (if measured) to the sweep's LDS slots: sums
// over each 16-lane row, one slot per (wave, row).
template <typename T, int W>
__device__ __forceinline__ void flush_partials(T *red, int d, bool meas, int wave, int wl, T &pe, T &pmx, T &pmy,
                                               T &pmz)
{
    if (d >= 0 && meas) {
        pe = row_sum(pe);
        pmx = row_sum(pmx);
        pmy = row_sum(pmy);
        pmz = row_sum(pmz);
        if ((wl & 15) == 0) {
            T *q = red + ((d * W + wave) * 4 + (wl >> 4)) * 4;
            q[0] += pe;
            q[1] += pmx;
            q[2] += pmy;
            q[3] += pmz;
        }
    }
    pe = pmx = pmy = pmz = T(0);
}

// Sweeps [k0, k1) of one path (the whole workgroup, B lanes) with spins in device memory
// (g.sp). win: LDS window of 4D + 4 plane slots; red: LDS [D][B/64 waves][4 rows][4]
// measurement partials.
template <typename T, int LC, int B, int D, bool GM>
__device__ __forceinline__ void path_sweeps_win(const GroupCtx<T> &g, const InstDev &in, int k0, int k1, bool fresh,
                                                T *win, T *red)
{
    constexpr int L = LC, HL = L / 2, PLANE = L * L / 2, SLOT = 6 * PLANE, NW = 4 * D + 4, W = B / 64;
    constexpr int HALF = L * PLANE;
    static_assert(L > 4 * D + 4, "the two copies of a plane must not meet in the window");
    const double Nd = (double)L * L * L;
    const int n_therm = in.n_therm, trace_sweeps = in.trace_sweeps, renorm_every = in.renorm_every;
    const double J = in.J;
    double *const trace = in.trace;
    Coef<T> cf;
    cf.beta = (T)in.beta;
    cf.J = (T)in.J;
    cf.q = (float)(in.beta * in.J * 1.4426950408889634);  // beta J log2(e)
    const int tid = g.lane, wave = tid >> 6, wl = tid & 63;
    unsigned long long nacc = 0;

    if (g.active && fresh) init_path<T, B>(g.sp, nullptr, nullptr, L, tid, g.path, g.key0, g.key1, g.ctr3, in.init);
    __syncthreads();
    for (int ks = k0; ks < k1;) {
        int Dp = k1 - ks < D ? k1 - ks : D;
        bool rn = false;
        if constexpr (std::is_same<T, float>::value) {
            if (renorm_every > 0) {
                const int next = (ks / renorm_every + 1) * renorm_every;
                if (next - ks < Dp) Dp = next - ks;
                rn = ks > 0 && ks % renorm_every == 0;
            }
        }
        const int NST = 2 * Dp;                 // stages of this pass
        const int vhi = L + NST - 1;            // last virtual plane read
        const int tau_end = 3 * (NST - 1) + L - 1;
        for (int i = tid; i < D * W * 16; i += B) red[i] = T(0);
        PlaneRegs<T, LC, B> cur;  // the plane stored into the window at the end of the step
        T pe = T(0), pmx = T(0), pmy = T(0), pmz = T(0);  // this wave's partials of sweep acc_d
        int acc_d = -1;
        bool acc_meas = false;
        if constexpr (GM) {
            // planes stay in device memory: normalise the whole lattice before the pass
            if constexpr (std::is_same<T, float>::value) {
                if (rn && g.active) renorm_path<B>(g.sp, nullptr, nullptr, L, tid);
            }
        } else if (g.active) {
#pragma unroll 1
            for (int v = -1; v <= 2; ++v) {
                PlaneRegs<T, LC, B> r;
                plane_load<T, LC, B>(r, g.sp, wrap_mod(v, L), tid, rn);
                plane_to_lds<T, LC, B>(r, win + wrap_mod(v, NW) * SLOT, tid);
            }
            plane_load<T, LC, B>(cur, g.sp, 3, tid, rn);
        }
        __syncthreads();
#pragma unroll 1
        for (int tau = 0; tau <= tau_end; ++tau) {
            // the plane whose last use was the previous step goes back to device memory
            const int vout = tau - 2 * NST;
            if (!GM && vout >= 0 && g.active)
                plane_writeback<T, LC, B>(win + wrap_mod(vout, NW) * SLOT, g.sp, wrap_mod(vout, L), tid);
            // prefetch of the plane first used four steps later (stored into the window next step)
            const int vin = tau + 3, vnext = tau + 4;
            const bool have_in = !GM && vin <= vhi && g.active;
            PlaneRegs<T, LC, B> nxt;
            if (!GM && vnext <= vhi && g.active) plane_load<T, LC, B>(nxt, g.sp, wrap_mod(vnext, L), tid, rn && vnext < L);
            // a sweep whose odd stage ended two steps ago is complete (its partials reached the
            // LDS slots at the start of the previous step): its measurement
            const int jf = tau - 2 - (L - 1);
            if (jf >= 3 && jf % 3 == 0 && ((jf / 3) & 1) && jf / 3 < NST) {
                const int d = (jf / 3) >> 1;
                const int k = ks + d;
                if ((k >= n_therm || k < trace_sweeps || k == k1 - 1) && g.active && wave == 0) {
                    T se = T(0), sx = T(0), sy = T(0), sz = T(0);
                    if (wl < 4 * W) {
                        const T *p = red + (d * W * 4 + wl) * 4;
                        se = p[0];
                        sx = p[1];
                        sy = p[2];
                        sz = p[3];
                    }
                    se = wave_sum(se);
                    sx = wave_sum(sx);
                    sy = wave_sum(sy);
                    sz = wave_sum(sz);
                    if (wl == 0) {
                        const double e = -J * (double)se / Nd;
                        const double mx = (double)sx / Nd, my = (double)sy / Nd, mz = (double)sz / Nd;
                        if (k >= n_therm) {
                            const double m = sqrt(mx * mx + my * my + mz * mz);
                            g.shacc[0] += e;
                            g.shacc[1] += e * e;
                            g.shacc[2] += m;
                            g.shacc[3] += m * m;
                            g.shacc[4] += (m * m) * (m * m);
                        }
                        if (k < trace_sweeps) {
                            double *tr = trace + ((size_t)g.path * trace_sweeps + k) * 4;
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
            }
            // active stages j: 3j <= tau < 3j + L; waves are dealt out over them
            int j_lo, j_hi, my, rank, nw;
            active_stages(tau, L, NST, j_lo, j_hi);
            deal_waves<2 * D>(wave, j_hi - j_lo + 1, W, my, rank, nw);
            my = __builtin_amdgcn_readfirstlane(my);
            rank = __builtin_amdgcn_readfirstlane(rank);
            nw = __builtin_amdgcn_readfirstlane(nw);
            // the partials stay in registers while the wave keeps serving the same sweep; they
            // go to the sweep's LDS slots when it moves on to another one
            if (((j_lo + my) >> 1) != acc_d) {
                flush_partials<T, W>(red, acc_d, acc_meas, wave, wl, pe, pmx, pmy, pmz);
                acc_d = (j_lo + my) >> 1;
                acc_meas = ks + acc_d >= n_therm || ks + acc_d < trace_sweeps || ks + acc_d == k1 - 1;
            }
            const int stage = j_lo + my;
            const int v = tau - 2 * stage, c = stage & 1, d = stage >> 1;
            const int k = ks + d;
            const int zp = wrap_mod(v, L);
            // own / oth: this plane's spins of each colour; component stride CS; dm / dp: the
            // offsets of the z-1 / z+1 planes (window slots, or device-memory planes)
            constexpr int CS = GM ? HALF : PLANE;
            int dm, dp;
            T *own;
            const T *oth;
            if constexpr (GM) {
                dm = (wrap_mod(v - 1, L) - zp) * PLANE;
                dp = (wrap_mod(v + 1, L) - zp) * PLANE;
                own = g.sp + c * 3 * HALF + zp * PLANE;
                oth = g.sp + (1 - c) * 3 * HALF + zp * PLANE;
            } else {
                const int sv = wrap_mod(v, NW);
                dm = (wrap_mod(v - 1, NW) - sv) * SLOT;
                dp = (wrap_mod(v + 1, NW) - sv) * SLOT;
                own = win + sv * SLOT + c * 3 * PLANE;
                oth = win + sv * SLOT + (1 - c) * 3 * PLANE;
            }
            if (g.active) {
#pragma unroll 2
                for (int s = rank * 64 + wl; s < PLANE; s += nw * 64) {
                    const int jx = s % HL, y = s / HL;
                    const int p = (y + zp + c) & 1;
                    Site st;
                    st.h = s;
                    st.id = 2 * jx + p + L * y + L * L * zp;
                    st.nb[0] = s + (p ? 0 : (jx == 0 ? HL - 1 : -1));
                    st.nb[1] = s + (p ? (jx == HL - 1 ? -(HL - 1) : 1) : 0);
                    st.nb[2] = s + (y == 0 ? (L - 1) * HL : -HL);
                    st.nb[3] = s + (y == L - 1 ? -(L - 1) * HL : HL);
                    st.nb[4] = s + dm;
                    st.nb[5] = s + dp;
                    update_site<T>(g, own, oth, CS, c != 0, st, (uint32_t)k, cf, pe, pmx, pmy, pmz, nacc);
                }
            }
            if (have_in) plane_to_lds<T, LC, B>(cur, win + wrap_mod(vin, NW) * SLOT, tid);
            if constexpr (!GM) cur = nxt;
            __syncthreads();
        }
        // the last sweep's measurement (the loop reaches the completion step of every other
        // sweep), and the planes still in the window
        flush_partials<T, W>(red, acc_d, acc_meas, wave, wl, pe, pmx, pmy, pmz);
        __syncthreads();
        {
            const int d = Dp - 1, k = ks + d;
            if ((k >= n_therm || k < trace_sweeps || k == k1 - 1) && g.active && wave == 0) {
                T se = T(0), sx = T(0), sy = T(0), sz = T(0);
                if (wl < 4 * W) {
                    const T *p = red + (d * W * 4 + wl) * 4;
                    se = p[0];
                    sx = p[1];
                    sy = p[2];
                    sz = p[3];
                }
                se = wave_sum(se);
                sx = wave_sum(sx);
                sy = wave_sum(sy);
                sz = wave_sum(sz);
                if (wl == 0) {
                    const double e = -J * (double)se / Nd;
                    const double mx = (double)sx / Nd, my = (double)sy / Nd, mz = (double)sz / Nd;
                    if (k >= n_therm) {
                        const double m = sqrt(mx * mx + my * my + mz * mz);
                        g.shacc[0] += e;
                        g.shacc[1] += e * e;
                        g.shacc[2] += m;
                        g.shacc[3] += m * m;
                        g.shacc[4] += (m * m) * (m * m);
                    }
                    if (k < trace_sweeps) {
                        double *tr = trace + ((size_t)g.path * trace_sweeps + k) * 4;
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
        }
        if (!GM && g.active) {
#pragma unroll 1
            for (int v = tau_end + 1 - 2 * NST; v <= L + NST - 2; ++v)
                plane_writeback<T, LC, B>(win + wrap_mod(v, NW) * SLOT, g.sp, wrap_mod(v, L), tid);
        }
        __syncthreads();
        ks += Dp;
    }
    if (g.active && wl == 0) atomicAdd((unsigned long long *)&g.shacc[9], nacc);
    __syncthreads();
}

// One path per workgroup (B lanes), spins in device memory at gsp, window in LDS (GM: the
// planes stay in device memory, LDS holds only the measurement partials).
template <typename T, int LC, int B, int D, bool GM>
__device__ __forceinline__ void wg_run_win(const InstDev &in, int path, int k0, int k1, bool fresh, char *smem, T *gsp)
{
    constexpr int NW = GM ? 0 : 4 * D + 4;
    GroupCtx<T> g;
    g.L = in.L;
    g.lane = threadIdx.x;
    g.path = (uint32_t)__builtin_amdgcn_readfirstlane(path);
    g.key0 = in.key0;
    g.key1 = in.key1;
    g.ctr3 = in.ctr3;
    g.active = path < in.n_paths;
    T *win = reinterpret_cast<T *>(smem);
    char *p = smem + (size_t)NW * 3 * LC * LC * sizeof(T);
    g.shacc = reinterpret_cast<double *>(p);
    T *red = reinterpret_cast<T *>(p + 128);
    g.red = red;
    g.sp = gsp;
    load_acc(g.shacc, in.acc + g.path, fresh, g.lane, g.active);
    path_sweeps_win<T, LC, B, D, GM>(g, in, k0, k1, fresh, win, red);
    store_acc(g.shacc, in.acc + g.path, g.lane, g.active);
}

template <typename T, int B, int D, bool GM>
constexpr int win_waves(int L)
{
    const int wgs = (int)((size_t)160 * 1024 / win_lds_bytes<T>(L, B, D, GM));
    const int cap = sizeof(T) == 8 ? 2 : (GM ? 4 : 8);
    const int w = (wgs < 1 ? 1 : wgs) * (B / 64) / 4;
    return w < 1 ? 1 : (w > cap ? cap : w);
}

template <typename T, int LC, int B, int D, bool GM>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(win_waves<T, B, D, GM>(LC))))
void k_window(InstDev in, int k0, int k1, int fresh)
{
    extern __shared__ __align__(16) char smem[];
    const int path = blockIdx.x;
    wg_run_win<T, LC, B, D, GM>(in, path, k0, k1, fresh != 0, smem,
                                reinterpret_cast<T *>(in.spins) + (size_t)path * 3 * LC * LC * LC);
}

template <typename T, int LC, int B, int D, bool GM>
hipError_t launch_window(const InstDev &in, int k0, int k1, int fresh, hipStream_t s)
{
    hipLaunchKernelGGL((k_window<T, LC, B, D, GM>), dim3(in.n_paths), dim3(B), win_lds_bytes<T>(LC, B, D, GM), s, in,
                       k0, k1, fresh);
    return hipGetLastError();
}

// ------------------------------------------------------------------ persistent batch kernel
constexpr int BATCH_B = 512;

// Variant lists of the batch kernels: (type, L or 0 for any, lanes per path, block, site map,
// Place, name). Index = BatchDev::variant value. Device-memory variants run in the shared
// kernel, whose block is BATCH_B; an LDS variant has a kernel, and a block, of its own.
#define MMC_BATCH_VARIANTS_F32(X)                                 \
    X(float, 8, 64, 512, COLZ, PL_LDS, "f32-lds-L8-g64")              \
    X(float, 12, 256, 512, FLAT, PL_LDS, "f32-lds-L12-g256")          \
    X(float, 16, 512, 512, COLZ, PL_LDS, "f32-lds-L16-g512")          \
    X(float, 20, 512, 512, FLAT, PL_LDS, "f32-lds-L20-g512")          \
    X(float, 20, 1024, 1024, COLZ, PL_LDS, "f32-lds-L20-g1024")       \
    X(float, 0, 512, 512, FLAT, PL_LDS, "f32-lds-any-g512")           \
    X(float, 24, 1024, 1024, FLAT, PL_SPLIT, "f32-split-L24-g1024")   \
    X(float, 30, 1024, 1024, COLZ, PL_SPLIT, "f32-split-L30-g1024")   \
    X(float, 0, 1024, 1024, FLAT, PL_SPLIT, "f32-split-any-g1024")    \
    X(float, 32, 1024, 1024, COLZ, PL_SPLIT_XY, "f32-splitxy-L32-g1024") \
    X(float, 0, 1024, 1024, FLAT, PL_SPLIT_XY, "f32-splitxy-any-g1024") \
    X(float, 48, 1024, 1024, FLAT, PL_RING, "f32-ring-L48-g1024")     \
    X(float, 48, 768, 768, FLAT, PL_RING, "f32-ring-L48-g768")        \
    X(float, 32, 512, 512, FLAT, PL_RING, "f32-ring-L32-g512")        \
    X(float, 64, 1024, 1024, FLAT, PL_HRING, "f32-hring-L64-g1024")   \
    X(float, 48, 768, 768, FLAT, PL_RING2, "f32-ring2-L48-g768")      \
    X(float, 48, 1024, 1024, FLAT, PL_RING2, "f32-ring2-L48-g1024")   \
    X(float, 32, 512, 512, FLAT, PL_RING2, "f32-ring2-L32-g512")      \
    X(float, 24, 512, 512, FLAT, PL_MEM, "f32-hbm-L24-g512")          \
    X(float, 32, 512, 512, COLZ, PL_MEM, "f32-hbm-L32-g512")          \
    X(float, 48, 512, 512, FLAT, PL_MEM, "f32-hbm-L48-g512")          \
    X(float, 64, 512, 512, COLZ, PL_MEM, "f32-hbm-L64-g512")          \
    X(float, 0, 512, 512, FLAT, PL_MEM, "f32-hbm-any-g512")

#define MMC_BATCH_VARIANTS_F64(X)                                 \
    X(double, 8, 128, 512, COLZ, PL_LDS, "f64-lds-L8-g128")           \
    X(double, 12, 512, 512, FLAT, PL_LDS, "f64-lds-L12-g512")         \
    X(double, 0, 512, 512, FLAT, PL_LDS, "f64-lds-any-g512")          \
    X(double, 0, 512, 512, FLAT, PL_SPLIT, "f64-split-any-g512")      \
    X(double, 32, 512, 512, COLZ, PL_MEM, "f64-hbm-L32-g512")         \
    X(double, 0, 512, 512, FLAT, PL_MEM, "f64-hbm-any-g512")

// The persistent batch kernel of one variant: workgroups take (instance, path group) items
// of the variant from its queue until the queue is empty. One kernel per variant lets each
// be compiled for its own occupancy, as the single-instance kernels are: the device-memory
// variants need more registers than the LDS ones. (The host runs a batch's kernels side by
// side on streams forked from the context's stream, or starts the LDS ones after the
// device-memory kernel when they carry little of the work.)
template <typename T, int LC, int G, int B, int MAP, int PL>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(target_waves<T>(LC, B, G, PL))))
void k_batch(BatchDev bd)
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
        wg_run<T, LC, G, B, MAP, PL>(in, item.path0, 0, in.n_therm + in.n_meas, true, smem, slot, false);
    }
}

template <typename T, int LC, int G, int B, int MAP, int PL>
hipError_t launch_batch_v(const BatchDev &b, int grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_batch<T, LC, G, B, MAP, PL>), dim3(grid), dim3(B), lds, s, b);
    return hipGetLastError();
}

// The device-memory variants share one persistent kernel: their items form one queue, largest
// first across all of them, so the long items of the largest lattices start first and the
// short ones fill the tail (memory-bound work, where the shared register budget costs little).
template <typename T>
__global__ __launch_bounds__(BATCH_B) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_mem(BatchDev bd)
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
        const int v = bd.variant[item.inst];
        int idx = 0;
#define MMC_BATCH_MEM_CASE(TT, LC, G, B, MAP, PL, NAME)                                                      \
    if constexpr (std::is_same<T, TT>::value) {                                                              \
        if constexpr (PL == PL_MEM) {                                                                        \
            static_assert(B == BATCH_B, "the shared device-memory kernel has one block size");              \
            if (v == idx) wg_run<TT, LC, G, BATCH_B, MAP, PL_MEM>(in, item.path0, 0, total, true, smem, slot, false); \
        }                                                                                                    \
        ++idx;                                                                                               \
    }
        MMC_BATCH_VARIANTS_F32(MMC_BATCH_MEM_CASE)
        MMC_BATCH_VARIANTS_F64(MMC_BATCH_MEM_CASE)
#undef MMC_BATCH_MEM_CASE
    }
}

template <typename T>
hipError_t launch_batch_mem(const BatchDev &b, int grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_mem<T>, dim3(grid), dim3(BATCH_B), lds, s, b);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fused batch kernel
// One persistent kernel of FUSED_B-lane workgroups for a batch that mixes lattice sides: every
// item of every instance goes into one queue, largest first, and each workgroup runs an item
// with the code of the instance's member variant (the same lanes per path, site map and
// placement as the batch variant it is named after, so each path's results are the same bit
// for bit). Its LDS and spin slots are the largest any member in the batch needs; its
// registers the largest any member needs (four waves per SIMD).
constexpr int FUSED_B = 1024;

#define MMC_FUSED_MEMBERS_F32(X)                                   \
    X(float, 48, 1024, FLAT, PL_RING, "f32-ring-L48-g1024")         \
    X(float, 32, 1024, COLZ, PL_SPLIT_XY, "f32-splitxy-L32-g1024")  \
    X(float, 30, 1024, COLZ, PL_SPLIT, "f32-split-L30-g1024")       \
    X(float, 24, 1024, FLAT, PL_SPLIT, "f32-split-L24-g1024")       \
    X(float, 20, 1024, COLZ, PL_LDS, "f32-lds-L20-g1024")           \
    X(float, 16, 512, COLZ, PL_LDS, "f32-lds-L16-g512")             \
    X(float, 12, 256, FLAT, PL_LDS, "f32-lds-L12-g256")             \
    X(float, 8, 64, COLZ, PL_LDS, "f32-lds-L8-g64")

// One item of a fused batch with member code (out of line: each member is register-allocated on
// its own, not as one union of every member's live values). The LDS base and the spin slot
// arrive with their address spaces (LDS, global), as does the instance: through generic
// pointers the member's every access would be a flat one.
using LdsPtr = __attribute__((address_space(3))) char *;
template <typename T>
using GlobalPtr = __attribute__((address_space(1))) T *;

template <typename T, int LC, int G, int MAP, int PL>
__device__ __attribute__((noinline)) void fused_item(GlobalPtr<const InstDev> in1, int path0, int total, LdsPtr smem3,
                                                     GlobalPtr<T> slot1)
{
    wg_run<T, LC, G, FUSED_B, MAP, PL>(*(const InstDev *)in1, path0, 0, total, true, (char *)smem3, (T *)slot1, false);
}

template <typename T>
__global__ __launch_bounds__(FUSED_B) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_fused(BatchDev bd)
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
        const int m = bd.variant[item.inst];  // the instance's fused member (workgroup-uniform)
        int idx = 0;
#define MMC_FUSED_CASE(TT, LC, G, MAP, PL, NAME)                                                          \
    if constexpr (std::is_same<T, TT>::value) {                                                           \
        if (m == idx)                                                                                     \
            fused_item<TT, LC, G, MAP, PL>((GlobalPtr<const InstDev>)&in, item.path0, total, (LdsPtr)smem,     \
                                           (GlobalPtr<TT>)slot);                                               \
        ++idx;                                                                                            \
    }
        MMC_FUSED_MEMBERS_F32(MMC_FUSED_CASE)
#undef MMC_FUSED_CASE
    }
}

// ------------------------------------------------------------------ plain FP64 engine
// One thread per site of one colour, spins in device memory, one launch per half-sweep;
// the sweep index lives in device memory so one captured sweep can be replayed.
__global__ __launch_bounds__(256) void k_plain_init(InstDev in)
{
    const int L = in.L, HALF = L * L * L / 2;
    const int h = blockIdx.x * 256 + threadIdx.x;
    const int path = blockIdx.y;
    if (blockIdx.x == 0 && threadIdx.x < 16) reinterpret_cast<double *>(in.acc + path)[threadIdx.x] = 0.0;
    if (h >= HALF) return;
    double *sp = reinterpret_cast<double *>(in.spins) + (size_t)path * 6 * HALF;
    const int init = in.init == INIT_MIXED ? ((path & 1) ? INIT_ORDERED : INIT_SPHERE) : in.init;
    for (int c = 0; c < 2; ++c) {
        const Site s = flat_site(L, h, c);
        double x, y, z;
        if (init == INIT_ORDERED) {
            x = 0.0; y = 0.0; z = 1.0;
        } else {
            const Words w = philox4x32_10((uint32_t)s.id, 0u, (uint32_t)path, TAG_INIT | in.ctr3, in.key0, in.key1);
            if (init == INIT_ANGLES) Arith<double>::angles(w.w0, w.w1, x, y, z);
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
    const int L = in.L, HALF = L * L * L / 2;
    const int h = blockIdx.x * 256 + threadIdx.x;
    const int path = blockIdx.y;
    unsigned long long nacc = 0;
    if (h < HALF) {
        GroupCtx<double> g;
        g.L = L;
        g.path = (uint32_t)path;
        g.key0 = in.key0;
        g.key1 = in.key1;
        g.ctr3 = in.ctr3;
        g.active = true;
        g.lane = h;
        g.sp = reinterpret_cast<double *>(in.spins) + (size_t)path * 6 * HALF;
        Coef<double> cf;
        cf.beta = in.beta;
        cf.J = in.J;
        cf.q = 0.0f;
        double pe = 0.0, px = 0.0, py = 0.0, pz = 0.0;
        double *own = g.sp + (c ? 3 * HALF : 0);
        const double *oth = g.sp + (c ? 0 : 3 * HALF);
        const Site s = flat_site(L, h, c);
        const uint32_t k = (uint32_t)*k_dev;
        if (in.proposal == PROPOSAL_ANGLES)
            update_site<double, true>(g, own, oth, HALF, c != 0, s, k, cf, pe, px, py, pz, nacc);
        else
            update_site<double, false>(g, own, oth, HALF, c != 0, s, k, cf, pe, px, py, pz, nacc);
    }
    if ((threadIdx.x & 63) == 0 && nacc) atomicAdd(&in.acc[path].n_accept, nacc);
}

// One workgroup per path: measures the state after the sweep, accumulates, then (thread 0)
// advances the device sweep counter.
__global__ __launch_bounds__(256) void k_plain_measure(InstDev in, int *k_dev, int k_last)
{
    __shared__ double part[4][4];
    const int L = in.L, HALF = L * L * L / 2;
    const int path = blockIdx.x;
    const double *sp = reinterpret_cast<const double *>(in.spins) + (size_t)path * 6 * HALF;
    const int k = *k_dev;
    const bool meas = k >= in.n_therm || k < in.trace_sweeps || k == k_last;
    if (meas) {
        double se = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        for (int h = threadIdx.x; h < HALF; h += 256) {
            const Site s = flat_site(L, h, 1);
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

// ------------------------------------------------------------------ proposal step alone
// The unit vector each precision's Metropolis move proposes from a word pair (the same
// Arith<T> code the sweep kernels inline), for checks of the proposal step on its own.
template <typename T, bool ANG>
__global__ __launch_bounds__(256) void k_proposals(const uint32_t *w, long long n, double *xyz)
{
    for (long long t = blockIdx.x * 256ll + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
        T x, y, z;
        if constexpr (ANG) Arith<T>::angles(w[2 * t], w[2 * t + 1], x, y, z);
        else Arith<T>::sphere(w[2 * t], w[2 * t + 1], x, y, z);
        xyz[3 * t + 0] = (double)x;
        xyz[3 * t + 1] = (double)y;
        xyz[3 * t + 2] = (double)z;
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
#define MMC_RES(TT, LC, G, B, MAP, PL, NAME)                                                          \
    Variant{NAME, std::is_same<TT, double>::value ? 1 : 0, LC, (int)(PL), B, G,                       \
            (LC ? lds_layout_bytes<TT>(LC, B, G, PL) : 0), &launch_resident<TT, LC, G, B, MAP, PL>,            \
            (const void *)&k_resident<TT, LC, G, B, MAP, PL>, 0},

#define MMC_WIN(TT, LC, B, D, GM, NAME)                                                               \
    Variant{NAME, std::is_same<TT, double>::value ? 1 : 0, LC, 0, B, B, win_lds_bytes<TT>(LC, B, D, GM),      \
            &launch_window<TT, LC, B, D, GM>, (const void *)&k_window<TT, LC, B, D, GM>, D},

static const Variant k_variants[] = {
    // FP32, spins in LDS
    MMC_RES(float, 8, 64, 256, COLZ, PL_LDS, "f32-lds-L8-g64-b256")
    MMC_RES(float, 8, 128, 256, COLZ, PL_LDS, "f32-lds-L8-g128-b256")
    MMC_RES(float, 8, 256, 256, COLZ, PL_LDS, "f32-lds-L8-g256-b256")
    MMC_RES(float, 10, 256, 256, COLZ, PL_LDS, "f32-lds-L10-g256-b256")
    MMC_RES(float, 12, 128, 256, FLAT, PL_LDS, "f32-lds-L12-g128-b256")
    MMC_RES(float, 12, 256, 256, FLAT, PL_LDS, "f32-lds-L12-g256-b256")
    MMC_RES(float, 16, 256, 256, COLZ, PL_LDS, "f32-lds-L16-g256-b256")
    MMC_RES(float, 16, 512, 512, COLZ, PL_LDS, "f32-lds-L16-g512-b512")
    MMC_RES(float, 16, 1024, 1024, COLZ, PL_LDS, "f32-lds-L16-g1024-b1024")
    MMC_RES(float, 0, 256, 256, FLAT, PL_LDS, "f32-lds-any-g256-b256")
    // colour 0 in LDS, colour 1 in device memory
    MMC_RES(float, 24, 1024, 1024, FLAT, PL_SPLIT, "f32-split-L24-g1024-b1024")
    MMC_RES(float, 30, 1024, 1024, COLZ, PL_SPLIT, "f32-split-L30-g1024-b1024")
    MMC_RES(float, 0, 512, 512, FLAT, PL_SPLIT, "f32-split-any-g512-b512")
    // colour 0's x and y in LDS, the rest in device memory
    MMC_RES(float, 32, 1024, 1024, COLZ, PL_SPLIT_XY, "f32-splitxy-L32-g1024-b1024")
    MMC_RES(float, 0, 512, 512, FLAT, PL_SPLIT_XY, "f32-splitxy-any-g512-b512")
    // FP32, spins in device memory
    MMC_RES(float, 24, 512, 512, FLAT, PL_MEM, "f32-hbm-L24-g512-b512")
    MMC_RES(float, 32, 512, 512, COLZ, PL_MEM, "f32-hbm-L32-g512-b512")
    MMC_RES(float, 32, 1024, 1024, COLZ, PL_MEM, "f32-hbm-L32-g1024-b1024")
    MMC_RES(float, 48, 512, 512, FLAT, PL_MEM, "f32-hbm-L48-g512-b512")
    MMC_RES(float, 64, 512, 512, COLZ, PL_MEM, "f32-hbm-L64-g512-b512")
    MMC_RES(float, 64, 1024, 1024, COLZ, PL_MEM, "f32-hbm-L64-g1024-b1024")
    MMC_RES(float, 0, 512, 512, FLAT, PL_MEM, "f32-hbm-any-g512-b512")
    // FP32, spins in device memory, swept through a ring of z-planes in LDS
    MMC_RES(float, 48, 1024, 1024, FLAT, PL_RING, "f32-ring-L48-b1024")
    MMC_RES(float, 48, 768, 768, FLAT, PL_RING, "f32-ring-L48-b768")
    MMC_RES(float, 32, 512, 512, FLAT, PL_RING, "f32-ring-L32-b512")
    MMC_RES(float, 16, 256, 256, FLAT, PL_RING, "f32-ring-L16-b256")
    // FP32, colour 0 through a ring of z-planes in LDS, colour 1 in place in device memory
    MMC_RES(float, 64, 1024, 1024, FLAT, PL_HRING, "f32-hring-L64-b1024")
    MMC_RES(float, 64, 768, 768, FLAT, PL_HRING, "f32-hring-L64-b768")
    MMC_RES(float, 48, 1024, 1024, FLAT, PL_HRING, "f32-hring-L48-b1024")
    MMC_RES(float, 16, 256, 256, FLAT, PL_HRING, "f32-hring-L16-b256")
    // FP32, spins in device memory, two sweeps per pass through a ring of z-planes in LDS
    MMC_RES(float, 48, 768, 768, FLAT, PL_RING2, "f32-ring2-L48-b768")
    MMC_RES(float, 48, 1024, 1024, FLAT, PL_RING2, "f32-ring2-L48-b1024")
    MMC_RES(float, 32, 512, 512, FLAT, PL_RING2, "f32-ring2-L32-b512")
    MMC_RES(float, 16, 128, 128, FLAT, PL_RING2, "f32-ring2-L16-b128")
    // FP32, spins in device memory, z-pipelined window in LDS
    MMC_WIN(float, 24, 512, 2, false, "f32-win-L24-d2-b512")
    MMC_WIN(float, 24, 1024, 3, false, "f32-win-L24-d3-b1024")
    MMC_WIN(float, 30, 1024, 2, false, "f32-win-L30-d2-b1024")
    MMC_WIN(float, 32, 512, 2, false, "f32-win-L32-d2-b512")
    MMC_WIN(float, 32, 1024, 2, false, "f32-win-L32-d2-b1024")
    // FP32, spins in device memory, z-pipelined schedule with every plane in device memory
    // (reuse through the caches)
    MMC_WIN(float, 32, 1024, 2, true, "f32-gwin-L32-d2-b1024")
    MMC_WIN(float, 48, 1024, 1, true, "f32-gwin-L48-d1-b1024")
    MMC_WIN(float, 64, 1024, 1, true, "f32-gwin-L64-d1-b1024")
    // FP64, spins in LDS
    MMC_RES(double, 8, 64, 256, COLZ, PL_LDS, "f64-lds-L8-g64-b256")
    MMC_RES(double, 8, 256, 256, COLZ, PL_LDS, "f64-lds-L8-g256-b256")
    MMC_RES(double, 12, 256, 256, FLAT, PL_LDS, "f64-lds-L12-g256-b256")
    MMC_RES(double, 16, 512, 512, COLZ, PL_LDS, "f64-lds-L16-g512-b512")
    MMC_RES(double, 0, 256, 256, FLAT, PL_LDS, "f64-lds-any-g256-b256")
    MMC_RES(double, 0, 512, 512, FLAT, PL_SPLIT, "f64-split-any-g512-b512")
    MMC_RES(double, 0, 512, 512, FLAT, PL_SPLIT_XY, "f64-splitxy-any-g512-b512")
    // FP64, spins in device memory
    MMC_RES(double, 16, 512, 512, COLZ, PL_MEM, "f64-hbm-L16-g512-b512")
    MMC_RES(double, 32, 512, 512, COLZ, PL_MEM, "f64-hbm-L32-g512-b512")
    MMC_RES(double, 64, 1024, 1024, COLZ, PL_MEM, "f64-hbm-L64-g1024-b1024")
    MMC_RES(double, 0, 512, 512, FLAT, PL_MEM, "f64-hbm-any-g512-b512")
    // FP64, plane ring (small lattices: parity of its schedule with the oracle)
    MMC_RES(double, 12, 256, 256, FLAT, PL_RING, "f64-ring-L12-b256")
    MMC_RES(double, 16, 256, 256, FLAT, PL_RING, "f64-ring-L16-b256")
    MMC_RES(double, 16, 256, 256, FLAT, PL_HRING, "f64-hring-L16-b256")
    MMC_RES(double, 16, 128, 128, FLAT, PL_RING2, "f64-ring2-L16-b128")
    // FP64, window (small lattices: parity of the pipelined schedule with the oracle)
    MMC_WIN(double, 12, 256, 1, false, "f64-win-L12-d1-b256")
    MMC_WIN(double, 16, 256, 2, false, "f64-win-L16-d2-b256")
    MMC_WIN(double, 16, 256, 2, true, "f64-gwin-L16-d2-b256")
    MMC_WIN(double, 24, 512, 3, true, "f64-gwin-L24-d3-b512")
};
#undef MMC_RES
#undef MMC_WIN

const Variant *variants(int *count)
{
    *count = (int)(sizeof(k_variants) / sizeof(k_variants[0]));
    return k_variants;
}

// LDS variants: a persistent kernel each; device-memory variants: the shared one
// The kernel and launcher of a batch variant: its own kernel for an LDS variant, the shared
// device-memory kernel otherwise (chosen at compile time, so no unused kernel is built).
template <typename T, int LC, int G, int B, int MAP, int PL>
constexpr const void *batch_kernel_of()
{
    if constexpr (PL != PL_MEM) return (const void *)&k_batch<T, LC, G, B, MAP, PL>;
    else return (const void *)&k_batch_mem<T>;
}

template <typename T, int LC, int G, int B, int MAP, int PL>
constexpr auto batch_launcher_of()
{
    if constexpr (PL != PL_MEM) return &launch_batch_v<T, LC, G, B, MAP, PL>;
    else return &launch_batch_mem<T>;
}

#define MMC_BV(TT, LC, G, B, MAP, PL, NAME)                                                          \
    Variant{NAME, std::is_same<TT, double>::value ? 1 : 0, LC, (int)(PL), B, G,                      \
            (LC ? lds_layout_bytes<TT>(LC, B, G, PL) : 0), nullptr,                                    \
            batch_kernel_of<TT, LC, G, B, MAP, PL>(), 0, batch_launcher_of<TT, LC, G, B, MAP, PL>()},
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

size_t variant_lds_bytes(const Variant &v, int L)
{
    if (v.window) return v.lds_bytes;
    return v.fp64 ? lds_layout_bytes<double>(L, v.block, v.lanes, v.lds) : lds_layout_bytes<float>(L, v.block, v.lanes, v.lds);
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
    if (v[variant].lds == PL_LDS) return 0;  // (a split variant sweeps colour 1 in its slot)
    return (size_t)(v[variant].block / v[variant].lanes) * 3 * (size_t)L * L * L * (fp64 ? 8 : 4);
}

int batch_blocks_per_cu(int fp64, int variant, size_t lds)
{
    int n;
    const Variant *v = batch_variants(fp64, &n);
    int blocks = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, v[variant].kernel, v[variant].block, lds);
    return e == hipSuccess ? blocks : 0;
}

hipError_t launch_batch(const BatchDev &b, int fp64, int variant, int grid, size_t lds, hipStream_t s)
{
    int n;
    const Variant *v = batch_variants(fp64, &n);
    return v[variant].launch_batch(b, grid, lds, s);
}

// The fused kernel's members: (name, side, lanes per path, placement) in member order.
struct FusedMember {
    const char *name;
    int L, lanes, place;
};
#define MMC_FUSED_ROW(TT, LC, G, MAP, PL, NAME) FusedMember{NAME, LC, G, (int)(PL)},
static const FusedMember k_fused_f32[] = {MMC_FUSED_MEMBERS_F32(MMC_FUSED_ROW)};
#undef MMC_FUSED_ROW

int fused_member(int fp64, const char *batch_variant)
{
    if (fp64 || !batch_variant) return -1;
    const int n = (int)(sizeof(k_fused_f32) / sizeof(k_fused_f32[0]));
    for (int i = 0; i < n; ++i)
        if (strcmp(k_fused_f32[i].name, batch_variant) == 0) return i;
    return -1;
}

size_t fused_lds_bytes(int member)
{
    const FusedMember &f = k_fused_f32[member];
    return lds_layout_bytes<float>(f.L, FUSED_B, f.lanes, f.place);
}

size_t fused_slot_bytes(int member)
{
    const FusedMember &f = k_fused_f32[member];
    if (f.place == PL_LDS) return 0;
    return (size_t)(FUSED_B / f.lanes) * 3 * (size_t)f.L * f.L * f.L * sizeof(float);
}

int fused_paths_per_item(int member) { return FUSED_B / k_fused_f32[member].lanes; }

const char *fused_member_name(int member) { return k_fused_f32[member].name; }

int fused_member_like(int fp64, int L, int place)
{
    if (fp64) return -1;
    const int n = (int)(sizeof(k_fused_f32) / sizeof(k_fused_f32[0]));
    for (int i = 0; i < n; ++i)
        if (k_fused_f32[i].L == L &&
            (k_fused_f32[i].place == place || (place == PL_RING2 && k_fused_f32[i].place == PL_RING)))
            return i;  // (the one-sweep ring's spins and accept counts are the two-sweep ring's)
    return -1;
}

int fused_block() { return FUSED_B; }

int fused_blocks_per_cu(size_t lds)
{
    int blocks = 0;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void *)&k_batch_fused<float>, FUSED_B, lds);
    return e == hipSuccess ? blocks : 0;
}

hipError_t launch_fused(const BatchDev &b, int grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_fused<float>, dim3(grid), dim3(FUSED_B), lds, s, b);
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
    const Variant *is = ising_variants(&n);
    for (int i = 0; i < n; ++i) raise_lds_limit(is[i].kernel, max_lds);
    for (int fp64 = 0; fp64 < 2; ++fp64) {
        int nb;
        const Variant *bv = batch_variants(fp64, &nb);
        for (int i = 0; i < nb; ++i) raise_lds_limit(bv[i].kernel, max_lds);
    }
    raise_lds_limit((const void *)&k_batch_fused<float>, max_lds);
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

hipError_t proposal_vectors(int fp64, int angles, const uint32_t *w, long long n, double *xyz, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int grid = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    if (fp64 && angles) hipLaunchKernelGGL((k_proposals<double, true>), dim3(grid), dim3(256), 0, s, w, n, xyz);
    else if (fp64) hipLaunchKernelGGL((k_proposals<double, false>), dim3(grid), dim3(256), 0, s, w, n, xyz);
    else if (angles) hipLaunchKernelGGL((k_proposals<float, true>), dim3(grid), dim3(256), 0, s, w, n, xyz);
    else hipLaunchKernelGGL((k_proposals<float, false>), dim3(grid), dim3(256), 0, s, w, n, xyz);
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
