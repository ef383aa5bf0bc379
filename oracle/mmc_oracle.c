/*
 * mmc_oracle.c -- plain, slow, obviously correct FP64 CPU oracle for the multipath
 * Metropolis simulation of the classical O(3) Heisenberg model.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library. It shares no source with the HIP engine: its Philox,
 * lattice indexing, update rule and measurements are written here from the paper and
 * from the published Philox definition, independently of the GPU code.
 *
 * What it follows (paper = arXiv:1305.6758, Sec. 2 "Simulation"):
 *   - Hamiltonian, eq. (ham), Sec. 2.1: H = -(J/2) sum_n sum_lambda S_n . S_{n+lambda},
 *     lambda running over the nearest neighbours, J = 1 fixes the energy scale.
 *   - Spherical parametrisation of unit spins, Sec. 2.1.
 *   - Sec. 2.2: every simulation path (SP) starts from a random (infinite-temperature)
 *     state, is swept with single-spin Metropolis moves, and outputs
 *     {M^x, M^y, M^z, H} per lattice site from its final state; a lattice sweep (LS) is
 *     L^3 Metropolis attempts.
 *   - Sec. 2.2, eq. (MCAV) and the moments <M^k>: time-averaged per-path moments are
 *     accumulated here in FP64 (per-site energy e, |m|, e^2, m^2, m^4).
 *
 * Readings where the paper is silent (each one is listed with its reason in the design
 * notes of the repository):
 *   - proposal: a new spin drawn uniformly on the sphere, independent of the old one
 *     (cos(theta) uniform on (-1,1), phi uniform on [0, 2 pi)); optionally both angles
 *     uniform (theta uniform on (0, pi)), the parametrisation of Sec. 2.2's random start
 *     applied to the moves (without a Hastings correction its stationary law is the
 *     Boltzmann weight times the product of 1/sin(theta_i), an easy-axis bias);
 *   - acceptance: accept iff u < exp(-beta dE), beta = 1/T, k_B = 1, u in (0,1);
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 *     as easy as 1, 2, 3", SC'11), counter (site, sweep, path, tag | instance << 8),
 *     key (seed_lo, seed_hi); uniform u = (w + 1/2) 2^-32, or on request the FP32 engine's
 *     grid u = ((w >> 8) | 1) 2^-24 (same words, FP64 arithmetic);
 *   - sweep: checkerboard (colour (x+y+z) mod 2; colour 0 then colour 1, each in increasing
 *     site id) -- the GPU order; the paper's literal random-site sweep and a typewriter
 *     sweep are kept for statistical cross-checks;
 *   - measurement after every sweep k >= n_therm; the final-state output of Sec. 2.2 is
 *     taken after the last sweep.
 *
 * Geometry: d = 1, 2 or 3 dimensions, side L, periodic or open boundaries. Site id
 * i = x + L (y + L z), x fastest. With periodic boundaries and L = 2 the +1 and -1
 * neighbours coincide and the literal 2d-neighbour sum counts that site twice.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fused multiply-add, so the
 * arithmetic is exactly the one written below).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MMCO_PI 3.14159265358979323846

/* ------------------------------------------------------------------------------------
 * Philox4x32-10, from the published definition (Salmon et al., SC'11, Sec. 3 and 4):
 * state of four 32-bit words, key of two; one round multiplies words 0 and 2 by the
 * two round multipliers, takes the 64-bit products apart into high and low halves and
 * permutes:  (w0, w1, w2, w3) -> (hi(M1 w2) ^ w1 ^ k0, lo(M1 w2), hi(M0 w0) ^ w3 ^ k1,
 * lo(M0 w0)); between rounds the key is bumped by the Weyl constants. 10 rounds.
 * ---------------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void mmco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t w0 = ctr[0], w1 = ctr[1], w2 = ctr[2], w3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)w0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)w2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ w1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ w3 ^ k1;
        uint32_t n3 = lo0;
        w0 = n0; w1 = n1; w2 = n2; w3 = n3;
        if (round < 9) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
    }
    out[0] = w0; out[1] = w1; out[2] = w2; out[3] = w3;
}

/* Vectorised convenience for tests: n independent calls. */
void mmco_philox_many(int64_t n, const uint32_t *ctr /* [n][4] */, const uint32_t *key /* [n][2] */,
                      uint32_t *out /* [n][4] */)
{
    for (int64_t t = 0; t < n; ++t)
        mmco_philox4x32_10(ctr + 4 * t, key + 2 * t, out + 4 * t);
}

/* Uniform on (0,1), exact: (w + 1/2) 2^-32. Never 0, never 1. */
double mmco_uniform(uint32_t w)
{
    return ((double)w + 0.5) * (1.0 / 4294967296.0);
}

/* The FP32 engine's uniform, exact: ((w >> 8) | 1) 2^-24 -- the top 23 bits of the word and
 * a trailing one, an odd multiple of 2^-24 in (0, 1). Used when the oracle is asked for the
 * FP32 grid, to compare with the FP32 engine step by step (same uniforms, FP64 arithmetic). */
double mmco_uniform_fp32(uint32_t w)
{
    return (double)((w >> 8) | 1u) * (1.0 / 16777216.0);
}

enum { MMCO_TAG_INIT = 0, MMCO_TAG_MET = 1, MMCO_TAG_SITE = 2 };
enum { MMCO_SWEEP_CHECKERBOARD = 0, MMCO_SWEEP_RANDOM_SITE = 1, MMCO_SWEEP_TYPEWRITER = 2,
       MMCO_SWEEP_CHECKERBOARD_REVERSED = 3 };
enum { MMCO_INIT_SPHERE = 0, MMCO_INIT_ANGLES = 1, MMCO_INIT_ORDERED = 2, MMCO_INIT_MIXED = 3 };
enum { MMCO_PROPOSAL_SPHERE = 0, MMCO_PROPOSAL_ANGLES = 1 };

typedef struct {
    int dim;           /* 1, 2 or 3 */
    int L;             /* side length */
    int periodic;      /* 1: periodic, 0: open */
    double T;          /* temperature; +inf means beta = 0 */
    double J;          /* coupling */
    int n_therm;
    int n_meas;
    uint64_t seed;
    uint32_t instance; /* goes into counter word 3 above the tag byte */
    int sweep;         /* MMCO_SWEEP_* */
    int init;          /* MMCO_INIT_* */
    int trace_sweeps;  /* record (e_k, M_k) for sweeps k < trace_sweeps */
    int proposal;      /* MMCO_PROPOSAL_* */
    int uniforms;      /* MMCO_UNIFORMS_*: how a word becomes a uniform */
} mmco_params;

enum { MMCO_UNIFORMS_FP64 = 0, MMCO_UNIFORMS_FP32 = 1 };

static double uniform_of(int grid, uint32_t w)
{
    return grid == MMCO_UNIFORMS_FP32 ? mmco_uniform_fp32(w) : mmco_uniform(w);
}

typedef struct {
    double e_mean, e2_mean, absm_mean, m2_mean, m4_mean; /* per site, means over n_meas */
    double final_m[3], final_e;                          /* final state, per site */
    uint64_t n_accept;                                   /* accepted Metropolis moves */
} mmco_path_result;

/* Per-path state that can be carried across calls (resume). */
typedef struct {
    double *spins;    /* [N][3] in site-id order */
    int sweeps_done;
    double sum_e, sum_e2, sum_m, sum_m2, sum_m4;
    uint64_t n_accept;
} mmco_state;

static int64_t n_sites(const mmco_params *p)
{
    int64_t n = 1;
    for (int a = 0; a < p->dim; ++a) n *= p->L;
    return n;
}

int64_t mmco_n_sites(const mmco_params *p) { return n_sites(p); }

static void site_coords(const mmco_params *p, int64_t i, int c[3])
{
    c[0] = c[1] = c[2] = 0;
    for (int a = 0; a < p->dim; ++a) {
        c[a] = (int)(i % p->L);
        i /= p->L;
    }
}

static int64_t coords_site(const mmco_params *p, const int c[3])
{
    int64_t i = 0;
    for (int a = p->dim - 1; a >= 0; --a) i = i * p->L + c[a];
    return i;
}

/* Nearest neighbours of site i in the fixed order (-x, +x, -y, +y, -z, +z) restricted to
 * the first dim axes. With open boundaries a missing neighbour is -1. Returns 2*dim. */
int mmco_neighbors(const mmco_params *p, int64_t i, int64_t out[6])
{
    int c[3];
    site_coords(p, i, c);
    int k = 0;
    for (int a = 0; a < p->dim; ++a) {
        for (int s = -1; s <= 1; s += 2) {
            int d[3] = { c[0], c[1], c[2] };
            int v = c[a] + s;
            if (v < 0 || v >= p->L) {
                if (p->periodic) v = (v + p->L) % p->L;
                else { out[k++] = -1; continue; }
            }
            d[a] = v;
            out[k++] = coords_site(p, d);
        }
    }
    return k;
}

int mmco_colour(const mmco_params *p, int64_t i)
{
    int c[3];
    site_coords(p, i, c);
    return (c[0] + c[1] + c[2]) & 1;
}

/* Local field h_i = sum of neighbour spins, added in the neighbour order above:
 * h = ((((S_-x + S_+x) + S_-y) + S_+y) + S_-z) + S_+z. */
void mmco_local_field(const mmco_params *p, const double *spins, int64_t i, double h[3])
{
    int64_t nb[6];
    int k = mmco_neighbors(p, i, nb);
    h[0] = h[1] = h[2] = 0.0;
    int first = 1;
    for (int t = 0; t < k; ++t) {
        if (nb[t] < 0) continue;
        const double *s = spins + 3 * nb[t];
        if (first) { h[0] = s[0]; h[1] = s[1]; h[2] = s[2]; first = 0; }
        else { h[0] = h[0] + s[0]; h[1] = h[1] + s[1]; h[2] = h[2] + s[2]; }
    }
}

/* Total energy, eq. (ham) read literally: -(J/2) sum_i S_i . h_i. */
double mmco_energy(const mmco_params *p, const double *spins)
{
    int64_t N = n_sites(p);
    double acc = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double h[3];
        mmco_local_field(p, spins, i, h);
        const double *s = spins + 3 * i;
        acc += (s[0] * h[0] + s[1] * h[1]) + s[2] * h[2];
    }
    return -(p->J / 2.0) * acc;
}

/* Energy change of replacing S_i by snew: dE = -J (snew - S_i) . h_i. */
double mmco_delta_e(const mmco_params *p, const double *spins, int64_t i, const double snew[3])
{
    double h[3];
    mmco_local_field(p, spins, i, h);
    const double *s = spins + 3 * i;
    double dx = snew[0] - s[0], dy = snew[1] - s[1], dz = snew[2] - s[2];
    return -p->J * ((dx * h[0] + dy * h[1]) + dz * h[2]);
}

/* Unit vector from two words by the spherical parametrisation of Sec. 2.1:
 *   SPHERE: cos(theta) = z = 2 u0 - 1 uniform, phi = 2 pi u1 (uniform on the sphere);
 *   ANGLES: theta = pi u0, phi = 2 pi u1 (both angles uniform);
 *   ORDERED: (0, 0, 1). */
static void unit_vector_grid(uint32_t w0, uint32_t w1, int mode, int grid, double s[3])
{
    if (mode == MMCO_INIT_ORDERED) { s[0] = 0.0; s[1] = 0.0; s[2] = 1.0; return; }
    double u0 = uniform_of(grid, w0), u1 = uniform_of(grid, w1);
    double phi = 2.0 * MMCO_PI * u1;
    if (mode == MMCO_INIT_ANGLES) {
        double theta = MMCO_PI * u0;
        s[0] = sin(theta) * cos(phi);
        s[1] = sin(theta) * sin(phi);
        s[2] = cos(theta);
        return;
    }
    double z = 2.0 * u0 - 1.0;
    double r = sqrt(1.0 - z * z);
    s[0] = r * cos(phi);
    s[1] = r * sin(phi);
    s[2] = z;
}

void mmco_unit_vector(uint32_t w0, uint32_t w1, int mode, double s[3])
{
    unit_vector_grid(w0, w1, mode, MMCO_UNIFORMS_FP64, s);
}

/* n unit vectors from word pairs w[2t], w[2t+1] on either uniform grid (vectorised for tests). */
void mmco_unit_vectors(int64_t n, const uint32_t *w, int mode, int grid, double *out /* [n][3] */)
{
    for (int64_t t = 0; t < n; ++t) unit_vector_grid(w[2 * t], w[2 * t + 1], mode, grid, out + 3 * t);
}

/* Many proposals for moment tests: draw t uses Philox((t, 0, 0, TAG_MET), seed). */
void mmco_proposals(int64_t n, uint64_t seed, double *out /* [n][3] */)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (int64_t t = 0; t < n; ++t) {
        uint32_t ctr[4] = { (uint32_t)t, (uint32_t)(t >> 32), 0u, MMCO_TAG_MET }, w[4];
        mmco_philox4x32_10(ctr, key, w);
        mmco_unit_vector(w[0], w[1], MMCO_INIT_SPHERE, out + 3 * t);
    }
}

/* Metropolis test of Sec. 2.2 with the acceptance min(1, exp(-beta dE)): accept iff
 * u < exp(-beta dE). For dE <= 0 the right side is >= 1 > u, so downhill moves are always
 * taken; for beta = 0 every move is taken. */
int mmco_accept(double u, double dE, double beta)
{
    return u < exp(-beta * dE);
}

static double beta_of(const mmco_params *p)
{
    return isinf(p->T) ? 0.0 : 1.0 / p->T;
}

static void words(const mmco_params *p, uint32_t c0, uint32_t c1, uint32_t path, uint32_t tag,
                  uint32_t w[4])
{
    uint32_t key[2] = { (uint32_t)p->seed, (uint32_t)(p->seed >> 32) };
    uint32_t ctr[4] = { c0, c1, path, tag | (p->instance << 8) };
    mmco_philox4x32_10(ctr, key, w);
}

/* One Metropolis attempt at site i with proposal words (w0, w1) and acceptance word w2. */
static int metropolis_site(const mmco_params *p, double beta, double *spins, int64_t i,
                           const uint32_t w[4])
{
    double snew[3];
    unit_vector_grid(w[0], w[1], p->proposal == MMCO_PROPOSAL_ANGLES ? MMCO_INIT_ANGLES : MMCO_INIT_SPHERE,
                     p->uniforms, snew);
    double dE = mmco_delta_e(p, spins, i, snew);
    double u = uniform_of(p->uniforms, w[2]);
    if (mmco_accept(u, dE, beta)) {
        spins[3 * i + 0] = snew[0];
        spins[3 * i + 1] = snew[1];
        spins[3 * i + 2] = snew[2];
        return 1;
    }
    return 0;
}

/* Initial state of Sec. 2.2 (per site, Philox((i, 0, path, TAG_INIT))). MIXED: the set-up of
 * Sec. 3 with half of the paths from a random start and half from the ordered one -- paths
 * with an even index start uniformly on the sphere, odd ones ordered. */
void mmco_init_state(const mmco_params *p, uint32_t path, mmco_state *st)
{
    int64_t N = n_sites(p);
    int mode = p->init;
    if (mode == MMCO_INIT_MIXED) mode = (path & 1u) ? MMCO_INIT_ORDERED : MMCO_INIT_SPHERE;
    for (int64_t i = 0; i < N; ++i) {
        uint32_t w[4];
        words(p, (uint32_t)i, 0u, path, MMCO_TAG_INIT, w);
        unit_vector_grid(w[0], w[1], mode, p->uniforms, st->spins + 3 * i);
    }
    st->sweeps_done = 0;
    st->sum_e = st->sum_e2 = st->sum_m = st->sum_m2 = st->sum_m4 = 0.0;
    st->n_accept = 0;
}

/* One lattice sweep k (N attempts) in the chosen order. */
static void sweep(const mmco_params *p, uint32_t path, int k, mmco_state *st)
{
    double beta = beta_of(p);
    int64_t N = n_sites(p);
    uint32_t w[4];
    if (p->sweep == MMCO_SWEEP_CHECKERBOARD || p->sweep == MMCO_SWEEP_CHECKERBOARD_REVERSED) {
        for (int colour = 0; colour < 2; ++colour) {
            for (int64_t t = 0; t < N; ++t) {
                int64_t i = (p->sweep == MMCO_SWEEP_CHECKERBOARD) ? t : N - 1 - t;
                if (mmco_colour(p, i) != colour) continue;
                words(p, (uint32_t)i, (uint32_t)k, path, MMCO_TAG_MET, w);
                st->n_accept += metropolis_site(p, beta, st->spins, i, w);
            }
        }
    } else if (p->sweep == MMCO_SWEEP_TYPEWRITER) {
        for (int64_t i = 0; i < N; ++i) {
            words(p, (uint32_t)i, (uint32_t)k, path, MMCO_TAG_MET, w);
            st->n_accept += metropolis_site(p, beta, st->spins, i, w);
        }
    } else { /* MMCO_SWEEP_RANDOM_SITE: N attempts at sites chosen uniformly (Sec. 2.2) */
        for (int64_t j = 0; j < N; ++j) {
            words(p, (uint32_t)j, (uint32_t)k, path, MMCO_TAG_SITE, w);
            int64_t i = (int64_t)(((uint64_t)w[3] * (uint64_t)N) >> 32);
            st->n_accept += metropolis_site(p, beta, st->spins, i, w);
        }
    }
}

/* Per-site energy e = E/N and magnetisation vector M = (1/N) sum_i S_i of a state. */
void mmco_observe(const mmco_params *p, const double *spins, double *e, double m[3])
{
    int64_t N = n_sites(p);
    *e = mmco_energy(p, spins) / (double)N;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        sx += spins[3 * i + 0];
        sy += spins[3 * i + 1];
        sz += spins[3 * i + 2];
    }
    m[0] = sx / (double)N;
    m[1] = sy / (double)N;
    m[2] = sz / (double)N;
}

/* Advance a path from st->sweeps_done to sweep k_end (exclusive), measuring after every
 * sweep k >= n_therm; trace rows (e_k, Mx_k, My_k, Mz_k) for k < trace_sweeps go to
 * trace[k*4 .. k*4+3] when trace is not NULL. */
void mmco_advance(const mmco_params *p, uint32_t path, int k_end, mmco_state *st, double *trace)
{
    for (int k = st->sweeps_done; k < k_end; ++k) {
        sweep(p, path, k, st);
        int meas = k >= p->n_therm;
        int tr = trace && k < p->trace_sweeps;
        if (meas || tr) {
            double e, m[3];
            mmco_observe(p, st->spins, &e, m);
            if (meas) {
                double am = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
                st->sum_e += e;
                st->sum_e2 += e * e;
                st->sum_m += am;
                st->sum_m2 += am * am;
                st->sum_m4 += (am * am) * (am * am);
            }
            if (tr) {
                trace[4 * k + 0] = e;
                trace[4 * k + 1] = m[0];
                trace[4 * k + 2] = m[1];
                trace[4 * k + 3] = m[2];
            }
        }
        st->sweeps_done = k + 1;
    }
}

void mmco_finish(const mmco_params *p, const mmco_state *st, mmco_path_result *r)
{
    double nm = (double)p->n_meas;
    if (p->n_meas > 0) {
        r->e_mean = st->sum_e / nm;
        r->e2_mean = st->sum_e2 / nm;
        r->absm_mean = st->sum_m / nm;
        r->m2_mean = st->sum_m2 / nm;
        r->m4_mean = st->sum_m4 / nm;
    } else {
        r->e_mean = r->e2_mean = r->absm_mean = r->m2_mean = r->m4_mean = NAN;
    }
    mmco_observe(p, st->spins, &r->final_e, r->final_m);
    r->n_accept = st->n_accept;
}

/* Run paths [path_begin, path_end) to completion. trace: [n][trace_sweeps][4] or NULL;
 * spins_out: [n][N][3] final states or NULL. n_threads <= 0 uses the OpenMP default.
 * Paths are independent; each one runs serially. Returns 0, or -1 on bad arguments. */
int mmco_run_paths(const mmco_params *p, int path_begin, int path_end, mmco_path_result *out,
                   double *trace, double *spins_out, int n_threads)
{
    if (!p || p->dim < 1 || p->dim > 3 || p->L < 1 || path_end < path_begin || p->n_therm < 0 ||
        p->n_meas < 0 || !(p->T > 0.0))
        return -1;
    int64_t N = n_sites(p);
    int n = path_end - path_begin;
#ifdef _OPENMP
    /* a thread count for this call only (the process-wide default stays as it was) */
    const int nthr = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr)
#else
    (void)n_threads;
#endif
    for (int t = 0; t < n; ++t) {
        mmco_state st;
        st.spins = (double *)malloc(sizeof(double) * 3 * (size_t)N);
        uint32_t path = (uint32_t)(path_begin + t);
        mmco_init_state(p, path, &st);
        double *tr = trace ? trace + (size_t)t * 4 * (size_t)p->trace_sweeps : NULL;
        mmco_advance(p, path, p->n_therm + p->n_meas, &st, tr);
        mmco_finish(p, &st, out + t);
        if (spins_out) memcpy(spins_out + (size_t)t * 3 * (size_t)N, st.spins, sizeof(double) * 3 * (size_t)N);
        free(st.spins);
    }
    return 0;
}

/* Threads the OpenMP runtime would use (for reporting the CPU baseline). */
int mmco_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------
 * Two-dimensional Ising model (appendix "2D Ising model"): spins s = +-1 on an L x L
 * periodic square lattice, H = -J sum over bonds s_i s_j, the same multipath set-up as the
 * Heisenberg model (random start, checkerboard Metropolis sweeps, per-path outputs).
 *
 * Site id i = x + L y; colour c = (x + y) mod 2; j = floor(x / 2) indexes the site within its
 * row of colour c. Readings where the appendix is silent (listed in the design notes):
 *   - move: flip s_i; dE = 2 J s_i h_i with h_i the sum of the four neighbours; accept iff
 *     u < exp(-beta dE) (downhill and level moves always taken);
 *   - random numbers: one Philox4x32-10 call serves a "quad" of four consecutive sites of a
 *     row of one colour: quad jq = floor(j / 4) of row y of colour c has index
 *     q = c L Q + y Q + jq with Q = ceil((L/2) / 4) quads per row; sweep k of path p uses
 *     counter (q, k, p, TAG_ISING | instance << 8) and the site takes word j mod 4 as its
 *     uniform u = (w + 1/2) 2^-32 (rows whose length is not a multiple of four leave the
 *     spare words of their last quad unused);
 *   - random start: counter (q, 0, p, TAG_ISING_INIT | instance << 8), word j mod 4: s = +1
 *     when w < 2^31, else -1; ORDERED: all +1; MIXED: even paths random, odd paths ordered;
 *   - outputs: per sweep e = E/N and m = M/N (signed); the per-path means of e, e^2, |m|,
 *     m^2, m^4 over the measured sweeps; final_m = (m, 0, 0) and final_e of the last state.
 * ---------------------------------------------------------------------------------- */
enum { MMCO_TAG_ISING = 3, MMCO_TAG_ISING_INIT = 4 };

static int ising_quads_per_row(int L) { return (L / 2 + 3) / 4; }

/* Uniform word of site (x, y) at counter word 1 = k (k = 0 with tag INIT for the start). */
static uint32_t ising_word(int L, int x, int y, uint32_t k, uint32_t path, uint32_t tag, uint32_t instance,
                           uint64_t seed)
{
    int Q = ising_quads_per_row(L), c = (x + y) & 1, j = x >> 1;
    uint32_t q = (uint32_t)(c * L * Q + y * Q + (j >> 2));
    uint32_t ctr[4] = { q, k, path, tag | (instance << 8) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t w[4];
    mmco_philox4x32_10(ctr, key, w);
    return w[j & 3];
}

static int ising_field(int L, const int8_t *s, int x, int y)
{
    int xm = (x + L - 1) % L, xp = (x + 1) % L, ym = (y + L - 1) % L, yp = (y + 1) % L;
    return s[xm + L * y] + s[xp + L * y] + s[x + L * ym] + s[x + L * yp];
}

/* Exported for the pins: the start and one Metropolis attempt, exactly as the runs do them. */
int mmco_ising_init_spin(int L, int x, int y, uint32_t path, uint32_t instance, uint64_t seed)
{
    return ising_word(L, x, y, 0u, path, MMCO_TAG_ISING_INIT, instance, seed) < 0x80000000u ? 1 : -1;
}

int mmco_ising_accept(int L, int x, int y, uint32_t k, uint32_t path, uint32_t instance, uint64_t seed,
                      double beta, double J, int s_times_h)
{
    double dE = 2.0 * J * (double)s_times_h;
    double u = mmco_uniform(ising_word(L, x, y, k, path, MMCO_TAG_ISING, instance, seed));
    return u < exp(-beta * dE);
}

/* Paths [path_begin, path_end) of the Ising model; out[t] as for the Heisenberg runs (final_m
 * = (M/N, 0, 0)); trace[t][k][4] = (e_k, m_k, 0, 0) for k < trace_sweeps; spins_out[t][N]. */
int mmco_ising_run_paths(int L, double T, double J, int n_therm, int n_meas, uint64_t seed, uint32_t instance,
                         int init, int path_begin, int path_end, int trace_sweeps, mmco_path_result *out,
                         double *trace, int8_t *spins_out, int n_threads)
{
    if (L < 2 || (L & 1) || !(T > 0.0) || n_therm < 0 || n_meas < 0 || path_end < path_begin) return -1;
    const int N = L * L;
    const double beta = isinf(T) ? 0.0 : 1.0 / T;
    const int n = path_end - path_begin;
#ifdef _OPENMP
    /* a thread count for this call only (the process-wide default stays as it was) */
    const int nthr = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr)
#else
    (void)n_threads;
#endif
    for (int t = 0; t < n; ++t) {
        const uint32_t path = (uint32_t)(path_begin + t);
        int8_t *s = (int8_t *)malloc((size_t)N);
        int mode = init == MMCO_INIT_MIXED ? ((path & 1u) ? MMCO_INIT_ORDERED : MMCO_INIT_SPHERE) : init;
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x)
                s[x + L * y] = (int8_t)(mode == MMCO_INIT_ORDERED ? 1 : mmco_ising_init_spin(L, x, y, path, instance, seed));
        double sum_e = 0, sum_e2 = 0, sum_m = 0, sum_m2 = 0, sum_m4 = 0, e = 0, m = 0;
        uint64_t acc = 0;
        const int K = n_therm + n_meas;
        for (int k = 0; k < K; ++k) {
            for (int c = 0; c < 2; ++c)
                for (int y = 0; y < L; ++y)
                    for (int x = 0; x < L; ++x) {
                        if (((x + y) & 1) != c) continue;
                        int a = s[x + L * y] * ising_field(L, s, x, y);
                        if (mmco_ising_accept(L, x, y, (uint32_t)k, path, instance, seed, beta, J, a)) {
                            s[x + L * y] = (int8_t)-s[x + L * y];
                            ++acc;
                        }
                    }
            /* H = -(J/2) sum_i s_i h_i and M = sum_i s_i, from the definition */
            long long sh = 0, M = 0;
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    sh += s[x + L * y] * ising_field(L, s, x, y);
                    M += s[x + L * y];
                }
            e = -J * (double)(sh / 2) / (double)N;
            m = (double)M / (double)N;
            if (k >= n_therm) {
                double am = fabs(m);
                sum_e += e;
                sum_e2 += e * e;
                sum_m += am;
                sum_m2 += m * m;
                sum_m4 += (m * m) * (m * m);
            }
            if (trace && k < trace_sweeps) {
                double *r = trace + ((size_t)t * trace_sweeps + k) * 4;
                r[0] = e;
                r[1] = m;
                r[2] = 0.0;
                r[3] = 0.0;
            }
        }
        mmco_path_result *o = out + t;
        if (n_meas > 0) {
            o->e_mean = sum_e / n_meas;
            o->e2_mean = sum_e2 / n_meas;
            o->absm_mean = sum_m / n_meas;
            o->m2_mean = sum_m2 / n_meas;
            o->m4_mean = sum_m4 / n_meas;
        } else {
            o->e_mean = o->e2_mean = o->absm_mean = o->m2_mean = o->m4_mean = NAN;
        }
        if (K == 0) {
            long long sh = 0, M = 0;
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    sh += s[x + L * y] * ising_field(L, s, x, y);
                    M += s[x + L * y];
                }
            e = -J * (double)(sh / 2) / (double)N;
            m = (double)M / (double)N;
        }
        o->final_m[0] = m;
        o->final_m[1] = 0.0;
        o->final_m[2] = 0.0;
        o->final_e = e;
        o->n_accept = acc;
        if (spins_out) memcpy(spins_out + (size_t)t * N, s, (size_t)N);
        free(s);
    }
    return 0;
}
