"""Pins of the oracle's portfolio P&L and its Value-at-Risk / Conditional
Value-at-Risk estimators (Sec. VI-B.1): the premium against Black-Scholes,
VaR and CVaR of short calls on one lognormal asset against their closed
forms, the empirical definitions against brute force on small samples
(ties included), and the mean P&L of zero-strike calls on correlated
assets against the lognormal mean under the real-world drift."""
import math

import numpy as np
import pytest

import oracle
import synth
from closed_forms import bs_call, short_calls_var_cvar

SEED = synth.SEED


def test_premium_is_black_scholes():
    S0, sig = np.array([100.0, 80.0]), np.array([0.2, 0.35])
    m, q = np.array([0.9, 1.0, 1.2]), np.array([1.0, -2.0, 0.5])
    want = sum(qk * bs_call(s, mk * s, 0.03, v, 1.5)
               for s, v in zip(S0, sig) for mk, qk in zip(m, q))
    assert abs(oracle.portfolio_premium(S0, sig, m, q, 0.03, 1.5) - want) < 1e-11


@pytest.mark.parametrize("n_steps", [1, 12])
def test_short_calls_var_cvar_closed_form(n_steps):
    # Log-Euler is exact in law, so any step count gives lognormal S_T.
    S0, mu, sig, r, T, alpha = 100.0, 0.08, 0.2, 0.03, 1.0, 0.95
    m, q = [1.0, 1.1], [-1.0, -1.0]
    prem = oracle.portfolio_premium([S0], [sig], m, q, r, T)
    N = 1 << 20
    pnl = oracle.portfolio_pnl([S0], [sig], [mu], [[1.0]], m, q, r, T, n_steps, N, SEED)
    var, cvar, k, nt = oracle.var_cvar(pnl, alpha)
    cf_var, cf_cvar, f = short_calls_var_cvar(S0, mu, sig, T, [S0 * x for x in m], q, prem, alpha)
    se_q = math.sqrt(alpha * (1 - alpha) / N) / f
    assert abs(var - cf_var) < 4 * se_q, (var, cf_var, se_q)
    tail = np.sort(pnl)[:k - 1]
    se_c = tail.std(ddof=1) / math.sqrt(k - 1) + se_q
    assert abs(cvar - cf_cvar) < 4 * se_c, (cvar, cf_cvar, se_c)
    assert k == int(N * 0.05) + 1 and nt == k - 1


def brute_var_cvar(x, alpha):
    # VaR = -inf{ v in sample : #{x_i <= v} / N > 1 - alpha }, scanning all v.
    N = len(x)
    cands = sorted(v for v in x if sum(1 for y in x if y <= v) / N > 1 - alpha)
    v = cands[0]
    tail = [y for y in x if -y > -v]
    return -v, (-sum(tail) / len(tail) if tail else float("nan"))


@pytest.mark.parametrize("seed", range(6))
def test_empirical_definitions_by_brute_force(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(20, 60))
    x = rng.normal(size=N).round(1)        # rounding makes ties likely
    for alpha in (0.9, 0.95, 0.75):
        v, c, _, _ = oracle.var_cvar(x, alpha)
        bv, bc = brute_var_cvar(list(x), alpha)
        assert v == bv
        assert (math.isnan(c) and math.isnan(bc)) or abs(c - bc) < 1e-12


def test_zero_strike_mean_pnl_on_correlated_assets():
    # q = 1 call of strike 0 on each asset: PnL = sum_a (S_{T,a} - S0_a), whose
    # mean is sum_a S0_a (e^{mu_a T} - 1) whatever the correlation.
    d = 16
    sigma, corr, _ = synth.basket_market(d)
    L = oracle.cholesky(corr)
    S0 = np.linspace(50, 150, d)
    mu = np.linspace(-0.05, 0.12, d)
    N = 1 << 16
    pnl = oracle.portfolio_pnl(S0, sigma, mu, L, [0.0], [1.0], 0.02, 1.0, 8, N, SEED)
    want = float(np.sum(S0 * (np.exp(mu) - 1.0)))
    assert abs(pnl.mean() - want) < 4 * pnl.std(ddof=1) / math.sqrt(N)
