"""Pins of the TTS statistics against closed forms: the exponential law of the fastest clone
(Eq. 2 and its derivation in the SM), percentile and mean estimators of tau, and the
short-timeout posterior of tau (Section "Running with a short timeout")."""
from __future__ import annotations

import math

import numpy as np
import pytest
from scipy import integrate

from paper_2102_09510_amd import tts_stats as ts


def test_percentile_closed_forms():
    assert ts.ttsp_from_tau(2.0, 99) == pytest.approx(2.0 * math.log(100.0))
    assert ts.ttsp_from_tau(3.0, 50) == pytest.approx(3.0 * math.log(2.0))
    assert ts.ttsp_from_tau(1.0, 90) == pytest.approx(math.log(10.0))


def test_estimators_on_exponential_samples():
    rng = np.random.default_rng(1)
    tau = 137.0
    x = rng.exponential(tau, size=40000)
    sd = tau / math.sqrt(x.size)
    assert abs(ts.tau_mean(x) - tau) < 4 * sd
    assert ts.tau_from_percentile(x, 50) == pytest.approx(tau, rel=0.03)
    assert ts.tau_from_percentile(x, 90) == pytest.approx(tau, rel=0.03)
    d, p = ts.ks_exponential(x, tau)
    assert p > 0.01 and d < 0.01
    d, p = ts.ks_exponential(rng.uniform(0, 2 * tau, size=4000), tau)
    assert p < 1e-6


def test_censored_mle():
    rng = np.random.default_rng(2)
    tau, cap = 50.0, 30.0
    x = rng.exponential(tau, size=50000)
    solved = x < cap
    est = ts.tau_censored_mle(np.minimum(x, cap), solved)
    assert est == pytest.approx(tau, rel=0.03)
    s = ts.summarize(x[solved], censored=int((~solved).sum()), cap=cap)
    assert s["tau"] == pytest.approx(est)


def test_fastest_of_many_clones_is_exponential():
    """SM derivation: single-clone times with p1(t) = 1 - t/t0 near 0 (here uniform on [0, t0])
    give a fastest-of-N_cl time that is exponential with tau = t0 / N_cl."""
    rng = np.random.default_rng(3)
    t0, ncl, runs = 1.0e6, 2000, 3000
    tts = np.array([rng.uniform(0, t0, size=ncl).min() for _ in range(runs)])
    tau = ts.tau_mean(tts)
    assert tau == pytest.approx(t0 / ncl, rel=0.06)
    assert ts.ks_exponential(tts, tau)[1] > 0.01
    assert ts.single_clone_scale(tau, ncl) == pytest.approx(t0, rel=0.06)


@pytest.mark.parametrize("n,n_run,t_max", [(5, 1000, 1.0), (20, 400, 2.5), (3, 50, 10.0)])
def test_inverse_gamma_posterior(n, n_run, t_max):
    post = ts.TimeoutPosterior(n, n_run, t_max)
    T = post.t_tot
    f = lambda u: float(post.pdf_inverse_gamma(u))
    total, _ = integrate.quad(f, 0, np.inf, limit=200)
    assert total == pytest.approx(1.0, rel=1e-6)
    if n > 1:
        m, _ = integrate.quad(lambda u: u * f(u), 0, np.inf, limit=200)
        assert m == pytest.approx(post.mean(), rel=1e-5)
    grid = np.linspace(T / (n + 20), T / max(n - 0.9, 0.1), 20001)
    assert grid[np.argmax(post.pdf_inverse_gamma(grid))] == pytest.approx(post.mode(), rel=1e-3)
    med = post.quantile(0.5)
    c, _ = integrate.quad(f, 0, med, limit=200)
    assert c == pytest.approx(0.5, abs=1e-6)


def test_exact_posterior_approaches_inverse_gamma_for_short_timeouts():
    """With t_max << tau the binomial posterior with the 1/tau prior and the inverse-gamma
    form agree (total variation small); with t_max comparable to tau they differ."""
    for t_max, tv_max in ((0.01, 0.02), (3.0, None)):
        post = ts.TimeoutPosterior(8, 800 if t_max < 1 else 10, t_max)
        T = post.t_tot
        grid = np.geomspace(T / 200, T * 5, 40001)
        le = post.log_exact(grid)
        pe = np.exp(le - le.max())
        pe /= np.trapezoid(pe, grid)
        pg = post.pdf_inverse_gamma(grid)
        tv = 0.5 * np.trapezoid(np.abs(pe - pg), grid)
        if tv_max is not None:
            assert tv < tv_max
        else:
            assert tv > 0.05


def test_shifted_exponential():
    rng = np.random.default_rng(4)
    x = 25.0 + rng.exponential(300.0, size=20000)
    loc, scale = ts.shifted_exponential(x)
    assert loc == pytest.approx(25.0, abs=0.5)
    assert scale == pytest.approx(300.0, rel=0.03)
    s = ts.summarize(x)
    assert s["shifted_ks_pvalue"] > 0.01


def test_tail_tau_ignores_early_times():
    """A law that is suppressed at short times but exponential beyond: the tail estimate
    recovers the scale, the plain mean does not."""
    rng = np.random.default_rng(5)
    x = rng.gamma(3.0, 40.0, size=30000)          # slow start
    x = np.where(x > 150, 150 + rng.exponential(200.0, size=x.size), x)
    tau, used = ts.tail_tau(x, 400.0)
    assert tau == pytest.approx(200.0, rel=0.05) and used > 1000
    assert abs(ts.tau_mean(x) - 200.0) > 20


def test_exact_timeout_posterior_quantiles():
    """The exact short-timeout posterior: its quantiles match the inverse-gamma form when
    t_max << tau, and a direct quadrature of the binomial-likelihood posterior otherwise."""
    import math


    q_ig = ts.TimeoutPosterior(10, 2000, 1e3)
    exact = ts.timeout_posterior_quantiles(10, 2000, 1e3)
    for q, v in zip((0.16, 0.5, 0.84), exact):
        assert abs(v / q_ig.quantile(q) - 1) < 0.01
    n, n_run, t_max = 9, 25, 1e6  # t_max / tau about 0.5: the inverse-gamma form is off
    post = ts.TimeoutPosterior(n, n_run, t_max)
    dens = lambda lt: math.exp(float(post.log_exact(math.exp(lt))) + lt + 60.0)
    lo, hi = math.log(t_max * 1e-2), math.log(t_max * 1e4)
    total = integrate.quad(dens, lo, hi, limit=400)[0]
    med = ts.timeout_posterior_quantiles(n, n_run, t_max, qs=(0.5,))[0]
    below = integrate.quad(dens, lo, math.log(med), limit=400)[0]
    assert abs(below / total - 0.5) < 0.005
    # near the binomial MLE tau = -t_max / ln(1 - n / n_run)
    mle = -t_max / math.log(1 - n / n_run)
    assert 0.8 < med / mle < 1.4
    with pytest.raises(ValueError):
        ts.timeout_posterior_quantiles(5, 5, 1.0)
