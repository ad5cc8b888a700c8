"""Closed and semi-closed forms used to pin the oracle.

These are textbook formulas, written independently of the oracle's path
simulation, so that a mistake in the oracle's dynamics, payoff or random
numbers shows up as a disagreement with them.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate
from scipy.stats import norm


# Black-Scholes-Merton (no dividends) -------------------------------------
def bs_call(S0, K, r, sigma, T):
    st = sigma * math.sqrt(T)
    d1 = (math.log(S0 / K) + (r + 0.5 * sigma * sigma) * T) / st
    d2 = d1 - st
    return S0 * norm.cdf(d1) - K * math.exp(-r * T) * norm.cdf(d2)


def bs_delta(S0, K, r, sigma, T):
    st = sigma * math.sqrt(T)
    d1 = (math.log(S0 / K) + (r + 0.5 * sigma * sigma) * T) / st
    return norm.cdf(d1)


def bs_vega(S0, K, r, sigma, T):
    st = sigma * math.sqrt(T)
    d1 = (math.log(S0 / K) + (r + 0.5 * sigma * sigma) * T) / st
    return S0 * norm.pdf(d1) * math.sqrt(T)


def lognormal_call(m, s2, K, disc):
    """disc * E[(e^Y - K)+] for Y ~ N(m, s2)."""
    s = math.sqrt(s2)
    d2 = (m - math.log(K)) / s
    d1 = d2 + s
    return disc * (math.exp(m + 0.5 * s2) * norm.cdf(d1) - K * norm.cdf(d2))


# Discretely sampled geometric-average Asian call (Kemna-Vorst type), average
# of ln S over the n dates t_i = i T/n, i = 1..n (S0 not included).
def geo_asian_call(S0, K, r, sigma, T, n):
    mu = r - 0.5 * sigma * sigma
    m = math.log(S0) + mu * T * (n + 1) / (2.0 * n)
    s2 = sigma * sigma * T * (n + 1) * (2 * n + 1) / (6.0 * n * n)
    return lognormal_call(m, s2, K, math.exp(-r * T))


# Continuously monitored up-and-out call, barrier H above the strike
# (Merton 1973; Reiner-Rubinstein 1991), no rebate.
def arith_asian2_call(S0, K, r, sigma, T):
    """Arithmetic-average Asian call on two fixings, S(T/2) and S(T), under
    GBM: e^{-rT} E[((S_1 + S_2)/2 - K)^+]. Given S_1 the inner expectation
    is a Black-Scholes call on S_2 / 2 over the second half with strike
    K - S_1 / 2 (or a forward when that strike is not positive); the outer
    expectation over the first half's normal is an adaptive quadrature."""
    dt = 0.5 * T
    sd = sigma * math.sqrt(dt)
    mu = (r - 0.5 * sigma * sigma) * dt

    def inner(z):
        a = 0.5 * S0 * math.exp(mu + sd * z)          # S_1 / 2
        fwd = a * math.exp(r * dt)                     # E[S_2 / 2 | S_1]
        kp = K - a
        if kp <= 0.0:
            v = a + fwd - K
        else:
            d1 = (math.log(a / kp) + (r + 0.5 * sigma * sigma) * dt) / sd
            v = fwd * norm.cdf(d1) - kp * norm.cdf(d1 - sd)
        return v * norm.pdf(z)

    # The integrand has a kink where K - S_1 / 2 changes sign.
    zk = (math.log(2.0 * K / S0) - mu) / sd
    lo, hi = -14.0, 14.0
    pts = [zk] if lo < zk < hi else None
    val, _ = integrate.quad(inner, lo, hi, points=pts, epsabs=1e-13, epsrel=1e-12, limit=400)
    return math.exp(-r * T) * val


def up_out_call(S, K, H, r, sigma, T):
    if S >= H:
        return 0.0
    if K >= H:
        return 0.0
    st = sigma * math.sqrt(T)
    mu = (r - 0.5 * sigma * sigma) / (sigma * sigma)
    x1 = math.log(S / K) / st + (1 + mu) * st
    x2 = math.log(S / H) / st + (1 + mu) * st
    y1 = math.log(H * H / (S * K)) / st + (1 + mu) * st
    y2 = math.log(H / S) / st + (1 + mu) * st
    df = math.exp(-r * T)
    A = S * norm.cdf(x1) - K * df * norm.cdf(x1 - st)
    Bt = S * norm.cdf(x2) - K * df * norm.cdf(x2 - st)
    p1 = (H / S) ** (2 * (mu + 1))
    p0 = (H / S) ** (2 * mu)
    Ct = S * p1 * norm.cdf(-y1) - K * df * p0 * norm.cdf(-y1 + st)
    Dt = S * p1 * norm.cdf(-y2) - K * df * p0 * norm.cdf(-y2 + st)
    return A - Bt + Ct - Dt


def bgk_discrete_up_out_call(S, K, H, r, sigma, T, n):
    """Broadie-Glasserman-Kou continuity correction for n monitoring dates."""
    beta1 = 0.5825971579390107  # -zeta(1/2)/sqrt(2*pi)
    return up_out_call(S, K, H * math.exp(beta1 * sigma * math.sqrt(T / n)), r,
                       sigma, T)


# Heston (1993) European call by Gil-Pelaez inversion of the characteristic
# function of ln S_T, in the rotation-safe form of Albrecher et al. (2007).
def heston_cf(u, S0, v0, kappa, theta, xi, rho, r, T):
    iu = 1j * u
    b = kappa - rho * xi * iu
    d = np.sqrt(b * b + xi * xi * (iu + u * u))
    g = (b - d) / (b + d)
    e = np.exp(-d * T)
    C = kappa * theta / (xi * xi) * ((b - d) * T - 2.0 * np.log((1 - g * e) / (1 - g)))
    D = (b - d) / (xi * xi) * (1 - e) / (1 - g * e)
    return np.exp(iu * (math.log(S0) + r * T) + C + D * v0)


def heston_call(S0, v0, kappa, theta, xi, rho, r, T, K):
    lnK = math.log(K)
    fwd = S0 * math.exp(r * T)

    def f2(u):
        return (np.exp(-1j * u * lnK) * heston_cf(u, S0, v0, kappa, theta, xi, rho, r, T)
                / (1j * u)).real

    def f1(u):
        return (np.exp(-1j * u * lnK) * heston_cf(u - 1j, S0, v0, kappa, theta, xi, rho, r, T)
                / (1j * u * fwd)).real

    opts = dict(limit=400, epsabs=1e-13, epsrel=1e-12)
    P1 = 0.5 + integrate.quad(f1, 1e-12, 200.0, **opts)[0] / math.pi
    P2 = 0.5 + integrate.quad(f2, 1e-12, 200.0, **opts)[0] / math.pi
    return S0 * P1 - K * math.exp(-r * T) * P2


def geo_basket_call(S0, sigma, corr, w, r, T, K):
    """disc * E[(exp(sum_a w_a ln S_T,a) - K)+] under correlated GBM."""
    S0 = np.asarray(S0, float)
    sigma = np.asarray(sigma, float)
    w = np.asarray(w, float)
    m = float(np.sum(w * (np.log(S0) + (r - 0.5 * sigma ** 2) * T)))
    ws = w * sigma
    s2 = float(ws @ np.asarray(corr) @ ws) * T
    return lognormal_call(m, s2, K, math.exp(-r * T))


# Risk metrics of a short-call position on one GBM asset (Sec. VI-B.1) -----
def short_calls_var_cvar(S0, mu, sigma, T, strikes, qty, premium, alpha):
    """VaR and CVaR of PnL = sum_k q_k (S_T - K_k)^+ - premium with all q_k < 0
    and S_T lognormal under drift mu: the P&L falls as S_T rises, so the loss
    tail is S_T above its alpha-quantile s. Requires s above every strike.
    Also returns the density of the P&L at its (1 - alpha)-quantile, for the
    standard error of the empirical quantile."""
    st = sigma * math.sqrt(T)
    z = norm.ppf(alpha)
    s = S0 * math.exp((mu - 0.5 * sigma * sigma) * T + st * z)
    assert all(q < 0 for q in qty) and s > max(strikes)
    pnl_s = sum(q * (s - K) for q, K in zip(qty, strikes)) - premium
    var = -pnl_s
    # E[S_T 1{S_T > s}] and P(S_T > s) = 1 - alpha
    d1 = (math.log(S0 / s) + (mu + 0.5 * sigma * sigma) * T) / st
    es = S0 * math.exp(mu * T) * norm.cdf(d1)
    tail = 1.0 - alpha
    cond = sum(q * (es - K * tail) for q, K in zip(qty, strikes)) / tail - premium
    cvar = -cond
    # density of S_T at s, mapped through |dPnL/dS| = -sum q_k
    fs = norm.pdf(z) / (s * st)
    f_pnl = fs / abs(sum(qty))
    return var, cvar, f_pnl


# European options with a continuous dividend yield q (Merton) -------------
def bs_call_div(S0, K, r, q, sigma, T):
    """Call on a stock paying dividend yield q: ln S_T ~ N(ln S0 + (r - q -
    sigma^2/2) T, sigma^2 T) under the pricing measure."""
    return lognormal_call(math.log(S0) + (r - q - 0.5 * sigma * sigma) * T, sigma * sigma * T,
                          K, math.exp(-r * T))


def bs_put_div(S0, K, r, q, sigma, T):
    """Put by put-call parity: P = C - S0 e^{-qT} + K e^{-rT}."""
    return bs_call_div(S0, K, r, q, sigma, T) - S0 * math.exp(-q * T) + K * math.exp(-r * T)


def max_call_independent(S0, sigma, r, q, T, K):
    """e^{-rT} E[(max(S_1, S_2) - K)+] for two independent lognormal assets
    with dividend yield q: E[(M - K)+] = int_K^inf P(M > x) dx and
    P(M > x) = 1 - F_1(x) F_2(x)."""
    def F(x, a):
        m = math.log(S0[a]) + (r - q - 0.5 * sigma[a] ** 2) * T
        return norm.cdf((math.log(x) - m) / (sigma[a] * math.sqrt(T)))
    v, _ = integrate.quad(lambda x: 1.0 - F(x, 0) * F(x, 1), K, np.inf, limit=400)
    return math.exp(-r * T) * v
