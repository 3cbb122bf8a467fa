"""Neuberger (Kenney-Laub) rational approximation of sign (test infrastructure only).

Section "Choice of the rational function":
  g_s(t) = ((t+1)^{2s} - (t-1)^{2s}) / ((t+1)^{2s} + (t-1)^{2s})      Eq. (neuberger_mit_c)
         = t sum_i omega_i / (t^2 - sigma_i)                          Eq. (pfe_s)
  omega_i = (1/s) cos^{-2}(pi (i - 1/2) / (2s)),  sigma_i = -tan^2(pi (i - 1/2) / (2s))
  sign(t) ~ g_s(c t)
Theorem (circle:thm): |g_s(t) - sign t| <= eps on the circle of centre
  M = (delta^2+1)/(delta^2-1) and radius R = 2 delta/(delta^2-1),
  delta = (2/eps + 1)^{1/(2s)}.
Choice of c and s for a spectrum inside C(m, r) u C(-m, r):
  c = ((m+r)(m-r))^{-1/2},  d = ((m+r)/(m-r))^{1/2},
  s >= log(eps/(eps+2)) / (2 log((d-1)/(d+1)))                        Eq. (no_of_poles)
Spectral-circle heuristic (numerical-results section): m = (alpha+beta)/2,
r = (beta-alpha)/2 from the smallest non-deflated modulus alpha and the
largest modulus beta.
Rescaled Neuberger (footnote on the choice of c): with e_max the largest
error of g_s(ct) on [alpha, beta], the factor 2/(2 - e_max) lowers it to
e_max/(2 - e_max).
Zolotarev's best rational approximation on [-beta,-alpha] u [alpha,beta]
(named there as the alternative for spectra close to the real axis), in the
standard form with Jacobi elliptic functions of modulus k' = sqrt(1 - k^2),
k = alpha/beta.
"""
from __future__ import annotations

import math

import numpy as np


def neuberger_pfe(s: int):
    """(omega, sigma) of Eq. (pfe_s), i = 1..s."""
    i = np.arange(1, s + 1, dtype=np.float64)
    th = np.pi / (2.0 * s) * (i - 0.5)
    omega = 1.0 / (s * np.cos(th) ** 2)
    sigma = -np.tan(th) ** 2
    return omega, sigma


def g_closed(s: int, t):
    """Closed form of Eq. (neuberger_mit_c)."""
    t = np.asarray(t, dtype=np.complex128)
    a = (t + 1.0) ** (2 * s)
    b = (t - 1.0) ** (2 * s)
    return (a - b) / (a + b)


def g_pfe(s: int, t):
    """Partial-fraction form of Eq. (pfe_s)."""
    t = np.asarray(t, dtype=np.complex128)
    om, sg = neuberger_pfe(s)
    return t * sum(w / (t * t - q) for w, q in zip(om, sg))


def circle(s: int, eps: float):
    """(centre M, radius R) of the circle C_{s,eps} of the circle theorem."""
    delta = (2.0 / eps + 1.0) ** (1.0 / (2 * s))
    return (delta ** 2 + 1) / (delta ** 2 - 1), 2 * delta / (delta ** 2 - 1)


def scale_from_circle(m: float, r: float):
    """(c, d) that map [m-r, m+r] onto [1/d, d]."""
    return ((m + r) * (m - r)) ** -0.5, ((m + r) / (m - r)) ** 0.5


def circle_from_extremes(alpha: float, beta: float):
    """(m, r) of the spectral-circle heuristic."""
    return 0.5 * (alpha + beta), 0.5 * (beta - alpha)


def poles_bound(alpha: float, beta: float, eps: float) -> float:
    """Right-hand side of Eq. (no_of_poles) (a real number)."""
    m, r = circle_from_extremes(alpha, beta)
    _, d = scale_from_circle(m, r)
    return math.log(eps / (eps + 2.0)) / (2.0 * math.log((d - 1.0) / (d + 1.0)))


def poles_needed(alpha: float, beta: float, eps: float) -> int:
    return int(math.ceil(poles_bound(alpha, beta, eps) - 1e-12))


def coefficients(s: int, alpha: float, beta: float):
    """(omega, sigma, c) for sign(t) ~ g_s(ct) on the circles through alpha, beta."""
    m, r = circle_from_extremes(alpha, beta)
    c, _ = scale_from_circle(m, r)
    om, sg = neuberger_pfe(s)
    return om, sg, c


def neuberger_rescaled(s: int, alpha: float, beta: float, npts: int = 200001):
    """(omega, sigma, c, e_max) of the rescaled Neuberger approximation: e_max is
    the largest |1 - g_s(ct)| over a dense grid of [alpha, beta] (g_s monotone on
    each side of ct = 1, so the grid includes both ends), omega scaled by
    2/(2 - e_max)."""
    om, sg, c = coefficients(s, alpha, beta)
    t = np.geomspace(alpha, beta, npts)
    e_max = float(np.max(np.abs(1.0 - g_closed(s, c * t).real)))
    return om * (2.0 / (2.0 - e_max)), sg, c, e_max


def zolotarev_product_coefficients(n: int, k: float):
    """c_1 .. c_{2n-1}: c_l = k^2 sn^2(l K'/(2n); k') / cn^2(l K'/(2n); k'),
    K' the complete elliptic integral of modulus k' = sqrt(1 - k^2)."""
    from scipy.special import ellipj, ellipk
    mp = 1.0 - k * k  # parameter (modulus squared) of k'
    Kp = float(ellipk(mp))
    l = np.arange(1, 2 * n, dtype=np.float64)
    sn, cn, _, _ = ellipj(l * Kp / (2 * n), mp)
    return k * k * sn ** 2 / cn ** 2


def zolotarev_unscaled(n: int, k: float, x):
    """x prod_{l<n} (x^2 + c_{2l}) / prod_{l<=n} (x^2 + c_{2l-1}) (no factor D)."""
    cc = zolotarev_product_coefficients(n, k)
    x = np.asarray(x, dtype=np.complex128)
    num = x.copy()
    den = np.ones_like(x)
    for l in range(1, n):
        num = num * (x * x + cc[2 * l - 1])
    for l in range(1, n + 1):
        den = den * (x * x + cc[2 * l - 2])
    return num / den


def zolotarev(n: int, alpha: float, beta: float, npts: int = 200001):
    """(omega, sigma, c, delta) with sign(t) ~ t' sum_i omega_i/(t'^2 - sigma_i), t' = c t,
    c = 1/beta; D = 2/(max + min) of the unscaled function over [k, 1], so that the
    error equioscillates between -delta and +delta, delta = (max-min)/(max+min).
    The extrema: a dense grid, the error of a provisional D split into runs of one
    sign, the largest deviation of each run refined by a bounded scalar search.
    The weights are D times the residues of the product form at x^2 = -c_{2i-1}."""
    from scipy.optimize import minimize_scalar
    k = alpha / beta
    cc = zolotarev_product_coefficients(n, k)
    odd = cc[0::2]   # c_1, c_3, ..., c_{2n-1}
    even = cc[1::2]  # c_2, ..., c_{2n-2}
    x = np.geomspace(k, 1.0, npts)
    f = zolotarev_unscaled(n, k, x).real
    e0 = 2.0 / (f.max() + f.min()) * f - 1.0
    cut = np.nonzero(np.sign(e0[1:]) != np.sign(e0[:-1]))[0] + 1
    vals = [f[0], f[-1]]
    for lo, hi in zip(np.concatenate(([0], cut)), np.concatenate((cut, [npts]))):
        j = lo + int(np.argmax(np.abs(e0[lo:hi])))
        sgn = -1.0 if e0[j] > 0 else 1.0  # maximise f on runs above 1, minimise below
        r = minimize_scalar(lambda u: sgn * zolotarev_unscaled(n, k, u).real,
                            bounds=(x[max(j - 1, 0)], x[min(j + 1, npts - 1)]), method="bounded",
                            options={"xatol": 1e-14 * x[j]})
        vals.append(zolotarev_unscaled(n, k, r.x).real)
    fmax, fmin = max(vals), min(vals)
    D = 2.0 / (fmax + fmin)
    delta = (fmax - fmin) / (fmax + fmin)
    a = np.empty(n)
    for i in range(n):
        num = np.prod(even - odd[i])
        den = np.prod(np.delete(odd, i) - odd[i])
        a[i] = num / den
    return D * a, -odd, 1.0 / beta, delta
