"""Cavity free energy of the K-spin model on a K-regular random hypergraph as a function of the
magnetisation, its spinodal temperature and the free-energy barrier that predicts the growth
rate of the time to solution (Section "Analytic prediction for exponent a in ln tau ~ a N").

Host-side numerics only. Variational free energy (Eq. (f)), with the readings fixed here:

    -beta f = log Z_i + log Z_a - K log Z_ai - beta b m
    Z_i  = 2 cosh(beta (K u + b)) / (2 cosh(beta u))^K
    Z_a  = cosh(beta) (1 + tanh(beta) tanh(beta h)^K)
    Z_ai = cosh(beta (u + h)) / (2 cosh(beta u) cosh(beta h))

stationary in (u, h, b) at
    m = tanh(beta (K u + b)),   h = (K - 1) u + b,   tanh(beta u) = tanh(beta) tanh(beta h)^(K-1).

The printed equation carries "+ K log Z_ai - b m"; with that sign the paramagnetic point
u = h = b = 0 would not give f_para = -log(2 cosh beta)/beta as the text states, so the cavity
(Bethe) form with -K log Z_ai and the Legendre term -beta b m is used. The spinodal is
1/T_sp = min_x atanh( tanh(x) / tanh((K-1) x)^(K-1) ): at b = 0 a ferromagnetic solution with
x = beta u needs tanh(beta) = tanh(x) / tanh((K-1) x)^(K-1); the printed product of the two
tanh factors has no minimum of that kind. Both readings reproduce the paper's numbers
(T_sp = 0.980548 and the barrier 0.0827249 at T_run = -2 / ln 0.055).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq, minimize_scalar


def t_run_from_w1(w1: float) -> float:
    """Pseudo-temperature of the quasi-greedy rule: w1 = exp(-2 / T_run) (Section "Numerical
    results")."""
    return -2.0 / math.log(w1)


def f_para(beta: float) -> float:
    """Paramagnetic free energy per spin, -log(2 cosh beta) / beta."""
    return -math.log(2.0 * math.cosh(beta)) / beta


def spinodal_temperature(K: int = 3) -> float:
    """T_sp: below it the ferromagnetic solution of the cavity equations exists."""
    g = lambda x: math.atanh(math.tanh(x) / math.tanh((K - 1) * x) ** (K - 1))
    r = minimize_scalar(g, bounds=(1e-6, 5.0), method="bounded",
                        options={"xatol": 1e-12, "maxiter": 500})
    return 1.0 / r.fun


def saddle_at_m(m: float, beta: float, K: int = 3) -> tuple[float, float, float]:
    """(u, h, b) solving the stationarity equations at fixed magnetisation m (0 < m < 1).

    With A = atanh(m) = beta (K u + b) and y = beta u, h = (A - y) / beta and
    tanh(y) = tanh(beta) tanh(A - y)^(K-1); the left side grows and the right side falls with y
    on [0, A], so the root is unique."""
    A = math.atanh(m)
    tb = math.tanh(beta)
    F = lambda y: math.tanh(y) - tb * math.tanh(A - y) ** (K - 1)
    y = brentq(F, 0.0, A, xtol=1e-15, rtol=1e-15, maxiter=500)
    u = y / beta
    h = (A - y) / beta
    b = A / beta - K * u
    return u, h, b


def beta_f_of_m(m: float, beta: float, K: int = 3) -> float:
    """beta f(m) from Eq. (f) at the saddle point with magnetisation m (m = 0: paramagnet)."""
    if m == 0.0:
        return beta * f_para(beta)
    u, h, b = saddle_at_m(m, beta, K)
    log_zi = math.log(2.0 * math.cosh(beta * (K * u + b))) - K * math.log(2.0 * math.cosh(beta * u))
    log_za = math.log(math.cosh(beta)) + math.log1p(math.tanh(beta) * math.tanh(beta * h) ** K)
    log_zai = (math.log(math.cosh(beta * (u + h))) - math.log(2.0)
               - math.log(math.cosh(beta * u)) - math.log(math.cosh(beta * h)))
    return -(log_zi + log_za - K * log_zai - beta * b * m)


def beta_delta_f(m: float, T: float, K: int = 3) -> float:
    """beta (f(m) - f_para) at temperature T."""
    beta = 1.0 / T
    return beta_f_of_m(m, beta, K) - beta * f_para(beta)


def barrier(T: float, K: int = 3, grid: int = 4000) -> tuple[float, float]:
    """(beta max_m Delta f, argmax m) between the paramagnet (m = 0) and the ferromagnetic
    minimum, for T below the spinodal: the free-energy barrier that sets tau ~ exp(N beta
    max Delta f)."""
    ms = np.linspace(1e-4, 1 - 1e-9, grid)
    vals = np.array([beta_delta_f(float(m), T, K) for m in ms])
    k = int(np.argmax(vals))
    lo, hi = ms[max(k - 1, 0)], ms[min(k + 1, grid - 1)]
    r = minimize_scalar(lambda m: -beta_delta_f(m, T, K), bounds=(lo, hi), method="bounded",
                        options={"xatol": 1e-13, "maxiter": 500})
    return -r.fun, float(r.x)
