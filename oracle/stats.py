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
  - Binder cumulant, eq. (kum): U_L = 1 - <M^4> / (3 <M^2>^2);
  - distribution coefficient, eq. (dist-coefficient), Sec. 3: least-squares line through
    the normal Q-Q plot, r = 1 - ||R||^2 / ((N-1) sigma^2);
  - coefficient of variation of the mean, eq. (eq:cv), Sec. 4.1: sigma_X / (sqrt(N) mean).
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
