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
