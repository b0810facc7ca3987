"""Pins of the cavity barrier calculator against the constants the paper prints and against
properties of the cavity solution."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2102_09510_amd import cavity as cv


def consts(golden):
    return {k: float(v[0][0]) for k, v in golden("cavity_constants.txt").items()}


def test_spinodal_temperature(golden):
    c = consts(golden)
    assert round(cv.spinodal_temperature(int(c["K"])), 6) == c["T_sp"]


def test_barrier_at_running_temperature(golden):
    c = consts(golden)
    T = cv.t_run_from_w1(c["w1"])
    assert T == pytest.approx(0.6896, abs=1e-4)  # "T_run ~ 0.69" in the text
    b, m_star = cv.barrier(T, int(c["K"]))
    assert round(b, 7) == c["barrier_at_T_run"]
    assert 0.0 < m_star < 1.0


def test_paramagnetic_limit_and_saddle_residuals():
    beta = 1.0 / 0.7
    assert cv.beta_f_of_m(0.0, beta) == pytest.approx(beta * cv.f_para(beta))
    assert cv.beta_delta_f(1e-5, 0.7) == pytest.approx(0.0, abs=1e-8)
    for m in (0.05, 0.4, 0.9, 0.999):
        u, h, b = cv.saddle_at_m(m, beta)
        assert math.tanh(beta * (3 * u + b)) == pytest.approx(m, rel=1e-10)
        assert h == pytest.approx(2 * u + b, rel=1e-10, abs=1e-12)
        assert math.tanh(beta * u) == pytest.approx(math.tanh(beta) * math.tanh(beta * h) ** 2,
                                                    rel=1e-9)


def test_stationarity_in_the_field():
    """At fixed m the variational free energy is stationary: perturbing u (and h, b through the
    constraints m and h = 2u + b) changes beta f only at second order."""
    beta, m, K = 1.0 / 0.75, 0.6, 3
    u, h, b = cv.saddle_at_m(m, beta, K)
    A = math.atanh(m)

    def bf(u_):
        b_ = A / beta - K * u_
        h_ = (K - 1) * u_ + b_
        lzi = math.log(2 * math.cosh(beta * (K * u_ + b_))) - K * math.log(2 * math.cosh(beta * u_))
        lza = math.log(math.cosh(beta)) + math.log1p(math.tanh(beta) * math.tanh(beta * h_) ** K)
        lzai = (math.log(math.cosh(beta * (u_ + h_))) - math.log(2)
                - math.log(math.cosh(beta * u_)) - math.log(math.cosh(beta * h_)))
        return -(lzi + lza - K * lzai - beta * b_ * m)

    e = 1e-4
    d1 = (bf(u + e) - bf(u - e)) / (2 * e)
    assert abs(d1) < 1e-6
    assert bf(u) == pytest.approx(cv.beta_f_of_m(m, beta, K), rel=1e-12)


def test_no_ferromagnetic_minimum_above_spinodal():
    """Above T_sp the free energy grows monotonically with m; below it a local minimum at large
    m appears, still above the paramagnet (no thermodynamic transition)."""
    ms = np.linspace(0.01, 0.999, 300)
    above = np.array([cv.beta_delta_f(float(m), 1.05) for m in ms])
    assert np.all(np.diff(above) > 0)
    below = np.array([cv.beta_delta_f(float(m), 0.7) for m in ms])
    k = int(np.argmax(below))
    assert 0 < k < ms.size - 1
    assert below[-1] < below[k] and below.min() >= -1e-9 and below[-1] > 0
