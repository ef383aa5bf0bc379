"""Cross-path statistics of the simulation output, FP64, written from their definitions.

TEST INFRASTRUCTURE: the oracle side of the statistics; the engine computes the same
quantities in its own host code.

Paper (arXiv:1305.6758):
  - MC average over paths, eq. (MCAV), eq. (M_and_H), Sec. 2.2;
  - moments <M^k> = <|M|^k>, k = 1, 2, 4, Sec. 2.2 (the printed |M| repeats M^x; the
    third term is read as (M^z)^2);
  - susceptibility and heat capacity, eq. (cv): chi = (L^3/T)(<M^2> - <M>^2),
    C_V = (L^3/T^2)(<H^2> - <H>^2); with per-path time averages the brackets are
    cross-path means of the per-path averaged moments;
  - Binder cumulant, eq. (kum): U_L = 1 - <M^4> / (3 <M^2>^2), with a first-order
    (delta-method) standard error from the cross-path covariance of (M^2, M^4);
  - critical temperature from the cumulant ratio, Sec. 4 (Fig. TCfig): U_L(Tc)/U_L'(Tc) = 1,
    the ratio taken linear in T between the two simulated temperatures;
  - distribution coefficient, eq. (dist-coefficient), Sec. 3: least-squares line through
    the normal Q-Q plot, r = 1 - ||R||^2 / ((N-1) sigma^2);
  - coefficient of variation of the mean, eq. (eq:cv), Sec. 3: sigma_X / (sqrt(N) mean).
Q-Q plotting positions (the paper does not name them): Filliben's order-statistic medians.
Normality p-value (the paper's Q-Q coefficient has no p-value): D'Agostino-Pearson K^2,
from D'Agostino (1970) for skewness, Anscombe & Glynn (1983) for kurtosis, and the
omnibus sum of squares with two degrees of freedom (D'Agostino, Belanger & D'Agostino 1990).
"""
import math

import numpy as np
from scipy.special import ndtri  # inverse standard normal CDF, used as a library primitive


def mean_se(x):
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    m = x.sum() / n
    var = ((x - m) ** 2).sum() / (n - 1) if n > 1 else float("nan")
    return m, math.sqrt(var / n)


def coeff_variation(x):
    """eq. (eq:cv): sigma_X / (sqrt(N) mean), sigma with n-1."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    m = x.sum() / n
    sd = math.sqrt(((x - m) ** 2).sum() / (n - 1))
    return sd / (math.sqrt(n) * m)


def filliben_medians(n):
    """Order-statistic medians of U(0,1) (Filliben 1975)."""
    m = np.empty(n)
    m[-1] = 0.5 ** (1.0 / n)
    m[0] = 1.0 - m[-1]
    i = np.arange(2, n)
    m[1:-1] = (i - 0.3175) / (n + 0.365)
    return m


def distribution_coefficient(x):
    """eq. (dist-coefficient): fit X_(i) = a + b q_i by least squares on the normal Q-Q
    plot (q_i = Phi^-1(m_i)); R_i = X_(i) - (a + b q_i); r = 1 - sum R_i^2/((N-1) s^2)."""
    x = np.sort(np.asarray(x, dtype=np.float64))
    n = x.size
    q = ndtri(filliben_medians(n))
    qm, xm = q.mean(), x.mean()
    b = ((q - qm) * (x - xm)).sum() / ((q - qm) ** 2).sum()
    a = xm - b * qm
    R = x - (a + b * q)
    s2 = ((x - xm) ** 2).sum() / (n - 1)
    return 1.0 - (R ** 2).sum() / ((n - 1) * s2)


def _z_skew(b1, n):
    y = b1 * math.sqrt((n + 1.0) * (n + 3.0) / (6.0 * (n - 2.0)))
    beta2 = (3.0 * (n * n + 27.0 * n - 70.0) * (n + 1.0) * (n + 3.0)
             / ((n - 2.0) * (n + 5.0) * (n + 7.0) * (n + 9.0)))
    w2 = -1.0 + math.sqrt(2.0 * (beta2 - 1.0))
    delta = 1.0 / math.sqrt(0.5 * math.log(w2))
    alpha = math.sqrt(2.0 / (w2 - 1.0))
    t = y / alpha
    return delta * math.log(t + math.sqrt(t * t + 1.0))


def _z_kurt(b2, n):
    e = 3.0 * (n - 1.0) / (n + 1.0)
    var = 24.0 * n * (n - 2.0) * (n - 3.0) / ((n + 1.0) ** 2 * (n + 3.0) * (n + 5.0))
    x = (b2 - e) / math.sqrt(var)
    sb1 = (6.0 * (n * n - 5.0 * n + 2.0) / ((n + 7.0) * (n + 9.0))
           * math.sqrt(6.0 * (n + 3.0) * (n + 5.0) / (n * (n - 2.0) * (n - 3.0))))
    A = 6.0 + 8.0 / sb1 * (2.0 / sb1 + math.sqrt(1.0 + 4.0 / (sb1 * sb1)))
    t1 = 1.0 - 2.0 / (9.0 * A)
    den = 1.0 + x * math.sqrt(2.0 / (A - 4.0))
    ratio = (1.0 - 2.0 / A) / den
    t2 = math.copysign(abs(ratio) ** (1.0 / 3.0), ratio)
    return (t1 - t2) / math.sqrt(2.0 / (9.0 * A))


def normality_k2(x):
    """D'Agostino-Pearson K^2 = Z(b1)^2 + Z(b2)^2 and its chi^2(2) p-value exp(-K^2/2).
    Needs n >= 20 for the kurtosis approximation."""
    x = np.asarray(x, dtype=np.float64)
    n = float(x.size)
    d = x - x.mean()
    m2 = (d ** 2).mean()
    m3 = (d ** 3).mean()
    m4 = (d ** 4).mean()
    b1 = m3 / m2 ** 1.5
    b2 = m4 / (m2 * m2)
    k2 = _z_skew(b1, n) ** 2 + _z_kurt(b2, n) ** 2
    return k2, math.exp(-0.5 * k2)


def binder_cumulant(m2, m4):
    """eq. (kum) and its standard error. U = 1 - A/(3 B^2) with A, B the cross-path means of
    the per-path M^4 and M^2 (independent paths). To first order in the fluctuations of the
    means, var U = (gA^2 s_AA + 2 gA gB s_AB + gB^2 s_BB)/n with gA = dU/dA = -1/(3 B^2),
    gB = dU/dB = 2A/(3 B^3) and s the sample (co)variances (n - 1)."""
    b = np.asarray(m2, dtype=np.float64)
    a = np.asarray(m4, dtype=np.float64)
    n = a.size
    A = a.sum() / n
    B = b.sum() / n
    U = 1.0 - A / (3.0 * B * B)
    ga = -1.0 / (3.0 * B * B)
    gb = 2.0 * A / (3.0 * B ** 3)
    da, db = a - A, b - B
    saa = (da * da).sum() / (n - 1)
    sbb = (db * db).sum() / (n - 1)
    sab = (da * db).sum() / (n - 1)
    var = (ga * ga * saa + 2.0 * ga * gb * sab + gb * gb * sbb) / n
    return U, math.sqrt(max(var, 0.0))


def cumulant_crossing(T1, T2, u, se):
    """Sec. 4: the temperature where U_L / U_L' = 1, with the ratio R(T) taken linear between
    T1 and T2. u = (U_L(T1), U_L'(T1), U_L(T2), U_L'(T2)) and se their standard errors, all four
    estimates independent. Returns (Tc, se_Tc, R1, se_R1, R2, se_R2).

    R_j = U_L(Tj)/U_L'(Tj), se(R_j) = |R_j| sqrt((se_L/U_L)^2 + (se_L'/U_L')^2);
    Tc = T1 + (1 - R1)(T2 - T1)/(R2 - R1), and to first order
    se(Tc) = |T2 - T1| sqrt(((1 - R2) se(R1))^2 + ((1 - R1) se(R2))^2) / (R2 - R1)^2."""
    R1 = u[0] / u[1]
    R2 = u[2] / u[3]
    s1 = abs(R1) * math.hypot(se[0] / u[0], se[1] / u[1])
    s2 = abs(R2) * math.hypot(se[2] / u[2], se[3] / u[3])
    dT = T2 - T1
    Tc = T1 + (1.0 - R1) * dT / (R2 - R1)
    sTc = abs(dT) * math.hypot((1.0 - R2) * s1, (1.0 - R1) * s2) / (R2 - R1) ** 2
    return Tc, sTc, R1, s1, R2, s2


def trace_statistics(trace, path_begin=0, path_stride=1):
    """Sec. 3 (Figs. TC_on_T, L10T1_T150_M_cv, ee): the order parameter <m> = <|M|> per site over
    paths and the coefficient of variation of that mean, eq. (eq:cv), after each sweep k; plus
    <e>. The state after sweep k of a path run longer is the final state of the same path run
    for k + 1 sweeps (same counters), so one traced run gives every sweep count at once.
    trace[p, k] = (e_k, Mx_k, My_k, Mz_k); paths path_begin, path_begin + stride, ...
    Returns rows (<m>, SE, cv, <e>, SE) per sweep."""
    t = np.asarray(trace, dtype=np.float64)[path_begin::path_stride]
    out = np.empty((t.shape[1], 5))
    for k in range(t.shape[1]):
        m = np.sqrt((t[:, k, 1:4] ** 2).sum(axis=1))
        out[k, 0], out[k, 1] = mean_se(m)
        out[k, 2] = coeff_variation(m)
        out[k, 3], out[k, 4] = mean_se(t[:, k, 0])
    return out


def path_statistics(res, L, T, dim=3):
    """Cross-path statistics of per-path results (dict of arrays as returned by
    oracle.run_paths)."""
    N = float(L ** dim)
    e = np.asarray(res["e_mean"])
    am = np.asarray(res["absm_mean"])
    n = e.size
    E, se_e = mean_se(e)
    M, se_m = mean_se(am)
    E2 = np.asarray(res["e2_mean"]).sum() / n
    M2 = np.asarray(res["m2_mean"]).sum() / n
    M4 = np.asarray(res["m4_mean"]).sum() / n
    out = {
        "n": n, "mean_e": E, "se_e": se_e, "mean_absm": M, "se_absm": se_m,
        "e2": E2, "m2": M2, "m4": M4,
        "chi": N / T * (M2 - M * M),
        "cv_heat": N / (T * T) * (E2 - E * E),
        "binder": 1.0 - M4 / (3.0 * M2 * M2),
    }
    if n >= 3:
        out["r_e"] = distribution_coefficient(e)
        out["r_absm"] = distribution_coefficient(am)
        out["cv_absm"] = coeff_variation(am)
    if n >= 20:
        out["p_norm_e"] = normality_k2(e)[1]
        out["p_norm_absm"] = normality_k2(am)[1]
    return out
