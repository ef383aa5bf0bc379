// stats.cpp -- host FP64 cross-path statistics of the simulation output
// (arXiv:1305.6758: eq. (MCAV), eq. (M_and_H), the moments <|M|^k>, eq. (cv), eq. (kum),
// eq. (dist-coefficient), eq. (eq:cv), and the cumulant-ratio crossing of Sec. 4).
#include <math.h>

#include <algorithm>
#include <vector>

#include "../../include/mmc.h"

namespace mmc {

// Inverse standard normal CDF, Wichura's algorithm AS241 (PPND16, Applied Statistics 37,
// 1988), relative accuracy about 1e-16.
double normal_quantile(double p)
{
    const double q = p - 0.5;
    if (fabs(q) <= 0.425) {
        const double r = 0.180625 - q * q;
        return q *
               (((((((2509.0809287301226727 * r + 33430.575583588128105) * r + 67265.770927008700853) * r +
                    45921.953931549871457) * r + 13731.693765509461125) * r + 1971.5909503065514427) * r +
                 133.14166789178437745) * r + 3.387132872796366608) /
               (((((((5226.495278852545925 * r + 28729.085735721942674) * r + 39307.89580009271061) * r +
                    21213.794301586595867) * r + 5394.1960214247511077) * r + 687.1870074920579083) * r +
                 42.313330701600911252) * r + 1.0);
    }
    double r = q < 0 ? p : 1.0 - p;
    if (r <= 0) return q < 0 ? -INFINITY : INFINITY;
    r = sqrt(-log(r));
    double val;
    if (r <= 5.0) {
        r -= 1.6;
        val = (((((((7.7454501427834140764e-4 * r + 0.0227238449892691845833) * r + 0.24178072517745061177) * r +
                   1.27045825245236838258) * r + 3.64784832476320460504) * r + 5.7694972214606914055) * r +
                4.6303378461565452959) * r + 1.42343711074968357734) /
              (((((((1.05075007164441684324e-9 * r + 5.475938084995344946e-4) * r + 0.0151986665636164571966) * r +
                   0.14810397642748007459) * r + 0.68976733498510000455) * r + 1.6763848301838038494) * r +
                2.05319162663775882187) * r + 1.0);
    } else {
        r -= 5.0;
        val = (((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r + 0.0012426609473880784386) * r +
                   0.026532189526576123093) * r + 0.29656057182850489123) * r + 1.7848265399172913358) * r +
                5.4637849111641143699) * r + 6.6579046435011037772) /
              (((((((2.04426310338993978564e-15 * r + 1.4215117583164458887e-7) * r + 1.8463183175100546818e-5) * r +
                   7.868691311456132591e-4) * r + 0.0148753612908506148525) * r + 0.13692988092273580531) * r +
                0.59983220655588793769) * r + 1.0);
    }
    return q < 0 ? -val : val;
}

// eq. (dist-coefficient): least-squares line through the normal Q-Q plot of x, at Filliben's
// order-statistic medians; r = 1 - sum(residual^2) / ((n - 1) s^2).
double distribution_coefficient(const std::vector<double> &x_in)
{
    const size_t n = x_in.size();
    if (n < 3) return NAN;
    std::vector<double> x(x_in);
    std::sort(x.begin(), x.end());
    std::vector<double> q(n);
    const double last = pow(0.5, 1.0 / (double)n);
    for (size_t i = 0; i < n; ++i) {
        double m;
        if (i == 0) m = 1.0 - last;
        else if (i == n - 1) m = last;
        else m = ((double)(i + 1) - 0.3175) / ((double)n + 0.365);
        q[i] = normal_quantile(m);
    }
    double qm = 0, xm = 0;
    for (size_t i = 0; i < n; ++i) {
        qm += q[i];
        xm += x[i];
    }
    qm /= (double)n;
    xm /= (double)n;
    double sqq = 0, sqx = 0, sxx = 0;
    for (size_t i = 0; i < n; ++i) {
        sqq += (q[i] - qm) * (q[i] - qm);
        sqx += (q[i] - qm) * (x[i] - xm);
        sxx += (x[i] - xm) * (x[i] - xm);
    }
    if (sxx == 0) return NAN;
    const double b = sqx / sqq, a = xm - b * qm;
    double rss = 0;
    for (size_t i = 0; i < n; ++i) {
        const double r = x[i] - (a + b * q[i]);
        rss += r * r;
    }
    return 1.0 - rss / sxx;  // (n - 1) s^2 = sum (x - mean)^2
}

// D'Agostino-Pearson omnibus test: K^2 = Z(b1)^2 + Z(b2)^2 with D'Agostino's (1970) skewness
// transform and Anscombe & Glynn's (1983) kurtosis transform; p = exp(-K^2 / 2) (chi^2, 2 dof).
double normality_p(const std::vector<double> &x)
{
    const double n = (double)x.size();
    if (x.size() < 20) return NAN;
    double mean = 0;
    for (double v : x) mean += v;
    mean /= n;
    double m2 = 0, m3 = 0, m4 = 0;
    for (double v : x) {
        const double d = v - mean;
        m2 += d * d;
        m3 += d * d * d;
        m4 += d * d * d * d;
    }
    m2 /= n;
    m3 /= n;
    m4 /= n;
    if (m2 == 0) return NAN;
    const double b1 = m3 / pow(m2, 1.5), b2 = m4 / (m2 * m2);
    // skewness
    const double y = b1 * sqrt((n + 1) * (n + 3) / (6.0 * (n - 2)));
    const double beta2 = 3.0 * (n * n + 27 * n - 70) * (n + 1) * (n + 3) / ((n - 2) * (n + 5) * (n + 7) * (n + 9));
    const double w2 = -1.0 + sqrt(2.0 * (beta2 - 1.0));
    const double delta = 1.0 / sqrt(0.5 * log(w2));
    const double alpha = sqrt(2.0 / (w2 - 1.0));
    const double t = y / alpha;
    const double z1 = delta * log(t + sqrt(t * t + 1.0));
    // kurtosis
    const double e = 3.0 * (n - 1) / (n + 1);
    const double var = 24.0 * n * (n - 2) * (n - 3) / ((n + 1) * (n + 1) * (n + 3) * (n + 5));
    const double xk = (b2 - e) / sqrt(var);
    const double sb1 = 6.0 * (n * n - 5 * n + 2) / ((n + 7) * (n + 9)) * sqrt(6.0 * (n + 3) * (n + 5) / (n * (n - 2) * (n - 3)));
    const double A = 6.0 + 8.0 / sb1 * (2.0 / sb1 + sqrt(1.0 + 4.0 / (sb1 * sb1)));
    const double t1 = 1.0 - 2.0 / (9.0 * A);
    const double ratio = (1.0 - 2.0 / A) / (1.0 + xk * sqrt(2.0 / (A - 4.0)));
    const double t2 = copysign(cbrt(fabs(ratio)), ratio);
    const double z2 = (t1 - t2) / sqrt(2.0 / (9.0 * A));
    return exp(-0.5 * (z1 * z1 + z2 * z2));
}

}  // namespace mmc

namespace mmc {

// Cross-path statistics of n path results of a lattice of N sites.
int stats_of(const mmc_path_result *res, int n, double N, double T, mmc_stats_t *out)
{
    if (!res || !out || n < 1 || !(N > 0) || !(T > 0)) return MMC_EINVAL;
    const double nd = (double)n;
    std::vector<double> e(n), m(n);
    double se = 0, sm = 0, se2 = 0, sm2 = 0, sm4 = 0, acc = 0;
    for (int i = 0; i < n; ++i) {
        e[i] = res[i].e_mean;
        m[i] = res[i].absm_mean;
        se += e[i];
        sm += m[i];
        se2 += res[i].e2_mean;
        sm2 += res[i].m2_mean;
        sm4 += res[i].m4_mean;
        acc += (double)res[i].n_accept;
    }
    mmc_stats_t s;
    s.n = n;
    s.mean_e = se / nd;
    s.mean_absm = sm / nd;
    double ve = 0, vm = 0;
    for (int i = 0; i < n; ++i) {
        ve += (e[i] - s.mean_e) * (e[i] - s.mean_e);
        vm += (m[i] - s.mean_absm) * (m[i] - s.mean_absm);
    }
    ve = n > 1 ? ve / (nd - 1) : NAN;
    vm = n > 1 ? vm / (nd - 1) : NAN;
    s.se_e = sqrt(ve / nd);
    s.se_absm = sqrt(vm / nd);
    s.e2 = se2 / nd;
    s.m2 = sm2 / nd;
    s.m4 = sm4 / nd;
    s.chi = N / T * (s.m2 - s.mean_absm * s.mean_absm);
    s.cv_heat = N / (T * T) * (s.e2 - s.mean_e * s.mean_e);
    s.binder = 1.0 - s.m4 / (3.0 * s.m2 * s.m2);
    s.cv_absm = sqrt(vm) / (sqrt(nd) * s.mean_absm);
    s.r_e = mmc::distribution_coefficient(e);
    s.r_absm = mmc::distribution_coefficient(m);
    s.p_norm_e = mmc::normality_p(e);
    s.p_norm_absm = mmc::normality_p(m);
    s.accept_rate = NAN;  // filled by callers that know the number of attempts
    (void)acc;
    *out = s;
    return MMC_OK;
}

}  // namespace mmc

extern "C" int mmc_stats_from_results(const mmc_path_result *res, int n, int L, double T, mmc_stats_t *out)
{
    if (L < 1) return MMC_EINVAL;
    return mmc::stats_of(res, n, (double)L * L * L, T, out);
}

extern "C" int mmc_binder_cumulant(const mmc_path_result *res, int n, double *U, double *se)
{
    if (!res || !U || !se || n < 2) return MMC_EINVAL;
    const double nd = (double)n;
    double A = 0, B = 0;
    for (int i = 0; i < n; ++i) {
        A += res[i].m4_mean;
        B += res[i].m2_mean;
    }
    A /= nd;
    B /= nd;
    double saa = 0, sbb = 0, sab = 0;
    for (int i = 0; i < n; ++i) {
        const double da = res[i].m4_mean - A, db = res[i].m2_mean - B;
        saa += da * da;
        sbb += db * db;
        sab += da * db;
    }
    saa /= nd - 1;
    sbb /= nd - 1;
    sab /= nd - 1;
    // first-order propagation: gradient of 1 - A/(3B^2) in (A, B)
    const double gA = -1.0 / (3.0 * B * B), gB = 2.0 * A / (3.0 * B * B * B);
    const double var = (gA * gA * saa + 2.0 * gA * gB * sab + gB * gB * sbb) / nd;
    *U = 1.0 - A / (3.0 * B * B);
    *se = sqrt(var > 0 ? var : 0.0);
    return MMC_OK;
}

extern "C" int mmc_cumulant_crossing(double T1, double T2, const double *u, const double *se, mmc_crossing_t *out)
{
    if (!u || !se || !out || !(T1 != T2)) return MMC_EINVAL;
    for (int i = 0; i < 4; ++i)
        if (!(u[i] != 0) || !isfinite(u[i]) || !(se[i] >= 0)) return MMC_EINVAL;
    mmc_crossing_t c;
    c.r_t1 = u[0] / u[1];
    c.r_t2 = u[2] / u[3];
    if (!(c.r_t2 != c.r_t1)) return MMC_EINVAL;
    c.se_r_t1 = fabs(c.r_t1) * hypot(se[0] / u[0], se[1] / u[1]);
    c.se_r_t2 = fabs(c.r_t2) * hypot(se[2] / u[2], se[3] / u[3]);
    // R linear in T: R(Tc) = 1
    const double slope = c.r_t2 - c.r_t1, dT = T2 - T1;
    c.tc = T1 + (1.0 - c.r_t1) * dT / slope;
    // dTc/dR1 = dT (1 - R2)/slope^2, dTc/dR2 = -dT (1 - R1)/slope^2
    c.se_tc = fabs(dT) * hypot((1.0 - c.r_t2) * c.se_r_t1, (1.0 - c.r_t1) * c.se_r_t2) / (slope * slope);
    *out = c;
    return MMC_OK;
}

extern "C" int mmc_distribution_coefficient(const double *x, int n, double *r)
{
    if (!x || !r || n < 3) return MMC_EINVAL;
    *r = mmc::distribution_coefficient(std::vector<double>(x, x + n));
    return MMC_OK;
}

extern "C" int mmc_trace_stats(const double *trace, int n_paths, int n_sweeps, int path_begin, int path_stride,
                               double *out)
{
    if (!trace || !out || n_sweeps < 1 || path_stride < 1 || path_begin < 0) return MMC_EINVAL;
    const int n = path_begin >= n_paths ? 0 : (n_paths - path_begin + path_stride - 1) / path_stride;
    if (n < 2) return MMC_EINVAL;
    const double nd = (double)n;
    for (int k = 0; k < n_sweeps; ++k) {
        double sm = 0, se = 0;
        for (int p = path_begin; p < n_paths; p += path_stride) {
            const double *r = trace + ((size_t)p * n_sweeps + k) * 4;
            sm += sqrt(r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
            se += r[0];
        }
        const double mm = sm / nd, me = se / nd;
        double vm = 0, ve = 0;
        for (int p = path_begin; p < n_paths; p += path_stride) {
            const double *r = trace + ((size_t)p * n_sweeps + k) * 4;
            const double dm = sqrt(r[1] * r[1] + r[2] * r[2] + r[3] * r[3]) - mm, de = r[0] - me;
            vm += dm * dm;
            ve += de * de;
        }
        vm /= nd - 1;
        ve /= nd - 1;
        double *o = out + (size_t)k * 5;
        o[0] = mm;
        o[1] = sqrt(vm / nd);
        o[2] = sqrt(vm) / (sqrt(nd) * mm);
        o[3] = me;
        o[4] = sqrt(ve / nd);
    }
    return MMC_OK;
}
