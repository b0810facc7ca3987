"""Time-to-solution statistics of many-clone runs (host-side, on the solver's outputs).

Section "Numerical results" and SM, "Derivation of the exponential distribution for the TTS":
with many clones the run's TTS (its fastest clone) is exponentially distributed,
P[TTS > t] = exp(-t / tau) (Eq. 2), with tau = t0 / N_cl where t0 is the single-clone scale. The
p-th percentile is TTS_p = -ln(1 - p/100) tau, so tau can be estimated from any percentile or,
better, from all runs (the mean).

Section "Running with a short timeout": N_run runs capped at t_max, n of them successful. The
posterior of tau under the scale-invariant prior 1/tau is proportional to
(1/tau) (1 - exp(-t_max/tau))^n exp(-t_max/tau)^(N_run - n); for t_max << tau it becomes the
inverse-gamma law with shape n and scale T_tot = N_run t_max.

Times can be in any unit (sweeps here); censored runs are those that reached the cap.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def ttsp_from_tau(tau: float, p: float) -> float:
    """TTS_p = -ln(1 - p/100) tau for the exponential law."""
    return -math.log1p(-p / 100.0) * tau


def tau_from_percentile(tts, p: float) -> float:
    """tau estimated from the empirical p-th percentile of uncensored TTS values."""
    return float(np.percentile(np.asarray(tts, dtype=float), p)) / -math.log1p(-p / 100.0)


def tau_mean(tts) -> float:
    """tau estimated as the mean TTS (maximum likelihood for uncensored exponential data)."""
    return float(np.mean(np.asarray(tts, dtype=float)))


def tau_censored_mle(times, solved) -> float:
    """Maximum-likelihood tau from runs that either solved at `times` or were censored there:
    total observed time over the number of successes."""
    t = np.asarray(times, dtype=float)
    s = np.asarray(solved, dtype=bool)
    if not s.any():
        return math.inf
    return float(t.sum() / s.sum())


def ks_exponential(tts, tau: float) -> tuple[float, float]:
    """Kolmogorov-Smirnov distance of the sample to the exponential law with scale tau and the
    asymptotic p-value (Kolmogorov distribution)."""
    x = np.sort(np.asarray(tts, dtype=float))
    n = x.size
    cdf = 1.0 - np.exp(-x / tau)
    i = np.arange(1, n + 1)
    d = float(max(np.max(i / n - cdf), np.max(cdf - (i - 1) / n)))
    # Kolmogorov series for P[sqrt(n) D > lam]
    lam = (math.sqrt(n) + 0.12 + 0.11 / math.sqrt(n)) * d
    pval = 2.0 * sum((-1) ** (k - 1) * math.exp(-2.0 * (k * lam) ** 2) for k in range(1, 101))
    return d, float(min(max(pval, 0.0), 1.0))


def shifted_exponential(tts) -> tuple[float, float]:
    """Maximum-likelihood location and scale of a shifted exponential, TTS = t_d + Exp(scale):
    t_d = the smallest TTS, scale = mean - t_d. A run cannot reach the ground state before the
    clones have descended from their random starts, so at small N the law starts after a delay;
    the paper's derivation (P[single clone not done] = 1 - t/t0 near t = 0) is its t_d -> 0
    limit."""
    x = np.asarray(tts, dtype=float)
    loc = float(x.min())
    return loc, float(x.mean() - loc)


def tail_tau(tts, t_c: float) -> tuple[float, int]:
    """tau of the exponential tail beyond t_c: for an exponential law the excess over any t_c is
    again exponential with the same scale (memorylessness), so mean(TTS - t_c | TTS > t_c)
    estimates it without the early-time part. Returns (tau, runs used)."""
    x = np.asarray(tts, dtype=float)
    tail = x[x > t_c] - t_c
    return (float(tail.mean()) if tail.size else math.inf), int(tail.size)


def single_clone_scale(tau: float, n_clones: int) -> float:
    """t0 = tau N_cl (SM): the scale that stays fixed when the clone count changes."""
    return tau * n_clones


@dataclass
class TimeoutPosterior:
    """Posterior of tau after n successes among n_run runs capped at t_max (Section "Running
    with a short timeout")."""
    n: int
    n_run: int
    t_max: float

    @property
    def t_tot(self) -> float:
        return self.n_run * self.t_max

    def log_exact(self, tau):
        """Unnormalised log posterior with the 1/tau prior and the binomial likelihood."""
        tau = np.asarray(tau, dtype=float)
        q = np.exp(-self.t_max / tau)
        return (-np.log(tau) + self.n * np.log1p(-q) + (self.n_run - self.n) * (-self.t_max / tau)
                + math.lgamma(self.n_run + 1) - math.lgamma(self.n + 1)
                - math.lgamma(self.n_run - self.n + 1))

    def pdf_inverse_gamma(self, tau):
        """The t_max << tau form: T^n / (n-1)! exp(-T/tau) / tau^(n+1)."""
        tau = np.asarray(tau, dtype=float)
        T, n = self.t_tot, self.n
        return np.exp(n * math.log(T) - math.lgamma(n) - T / tau - (n + 1) * np.log(tau))

    def mean(self) -> float:
        """Posterior mean of the inverse-gamma form, T/(n-1) (n > 1)."""
        return self.t_tot / (self.n - 1) if self.n > 1 else math.inf

    def mode(self) -> float:
        return self.t_tot / (self.n + 1)

    def quantile(self, q: float) -> float:
        """Quantile of the inverse-gamma form: tau = T / x with x the (1-q) quantile of the
        Gamma(n, 1) law, found by bisection on its regularised incomplete gamma function."""
        from scipy.special import gammaincc

        lo, hi = 1e-12, max(10.0, 10.0 * self.n)
        target = q  # P[tau <= T/x] = P[X >= x] = Q(n, x)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if gammaincc(self.n, mid) > target:
                lo = mid
            else:
                hi = mid
        return self.t_tot / (0.5 * (lo + hi))


def timeout_posterior_quantiles(n: int, n_run: int, t_max: float, qs=(0.16, 0.5, 0.84),
                                grid: int = 20000) -> list[float]:
    """Quantiles of the exact posterior of tau (binomial likelihood of n successes in n_run runs
    capped at t_max, prior 1/tau; Section "Running with a short timeout"), for any t_max/tau,
    by integration on a log grid of tau (the inverse-gamma form needs t_max << tau)."""
    if not 0 < n < n_run:
        raise ValueError("need 0 < n < n_run (with every run solved the 1/tau prior leaves "
                         "the posterior improper at small tau)")
    post = TimeoutPosterior(n, n_run, t_max)
    lo, hi = t_max * 1e-3, post.t_tot * 1e3
    lt = np.linspace(math.log(lo), math.log(hi), grid)
    tau = np.exp(lt)
    # density in log tau: p(tau) tau
    logd = post.log_exact(tau) + lt
    w = np.exp(logd - logd.max())
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return [float(np.exp(np.interp(q, cdf, lt))) for q in qs]


def summarize(tts, censored: int = 0, cap: float | None = None,
              n_clones: int | None = None) -> dict:
    """Estimates of tau from run TTS values; `censored` runs reached `cap` without a solution
    (their time enters the maximum-likelihood estimate). Adds the predicted and empirical
    TTS_99 and the exponential-law check of the solved runs."""
    tts = np.asarray(tts, dtype=float)
    out = {"runs": int(tts.size + censored), "solved": int(tts.size), "censored": int(censored)}
    if tts.size >= 2:
        if censored:
            if cap is None:
                raise ValueError("censored runs need the cap")
            tau = tau_censored_mle(np.r_[tts, np.full(censored, cap)],
                                   np.r_[np.ones(tts.size, bool), np.zeros(censored, bool)])
        else:
            tau = tau_mean(tts)
        out.update(tau=tau, tts99_from_tau=ttsp_from_tau(tau, 99))
        if not censored:
            out.update(tau_from_p50=tau_from_percentile(tts, 50),
                       tau_from_p90=tau_from_percentile(tts, 90),
                       tts99_empirical=float(np.percentile(tts, 99)))
            d, pv = ks_exponential(tts, tau)
            out.update(ks_distance=d, ks_pvalue=pv)
            t_c = float(np.percentile(tts, 50))
            tt, used = tail_tau(tts, t_c)
            dt_, pvt = ks_exponential(tts[tts > t_c] - t_c, tt)
            out.update(tail_from=t_c, tail_tau=tt, tail_runs=used, tail_ks_pvalue=pvt)
            if n_clones:
                out["t0_tail"] = single_clone_scale(tt, n_clones)
            loc, scale = shifted_exponential(tts)
            d2, pv2 = ks_exponential(tts - loc, scale)
            out.update(shifted_loc=loc, shifted_scale=scale, shifted_ks_distance=d2,
                       shifted_ks_pvalue=pv2)
            if n_clones:
                out["t0_shifted"] = single_clone_scale(scale, n_clones)
        if n_clones:
            out["t0"] = single_clone_scale(tau, n_clones)
    return out
