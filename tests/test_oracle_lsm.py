"""Pins of the oracle's Longstaff-Schwartz estimator (Sec. II-A.3, the
American max-option experiment of Sec. VI-C) and of the binomial lattice
that stands in for the true price:

* the lattice against Black-Scholes with dividends and against the exact
  one-dimensional integral of the two-asset max-call, Bermudan features
  that are exact on a lattice (no early exercise of a call on a
  dividend-free stock; the put's value rising with the number of dates),
  and the paper's quoted value for the max-call;
* each regression of the estimator against numpy's least squares on the
  in-the-money paths, with the cash flows rebuilt from its own decisions;
* the estimator against the lattice, its single-date and
  out-of-the-money degenerations, and the out-of-sample estimator with an
  inactive rule against the European payoff on the same paths.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from closed_forms import bs_call_div, bs_put_div, max_call_independent
from lsm_basis import features as _feat, payoff as _payoff

SEED = synth.SEED
HERE = os.path.dirname(os.path.abspath(__file__))
MAXC, PUT, CALL = oracle.LSM_MAX_CALL, oracle.LSM_BASKET_PUT, oracle.LSM_BASKET_CALL


# ---- the lattice -----------------------------------------------------------
@pytest.mark.parametrize("kind,closed", [(CALL, bs_call_div), (PUT, bs_put_div)])
def test_lattice_single_date_is_black_scholes(kind, closed):
    v = oracle.lsm_lattice([100.0], [0.25], 0.04, 0.03, 2.0, kind, 95.0, 1, 2000)
    assert abs(v - closed(100.0, 95.0, 0.04, 0.03, 0.25, 2.0)) < 2e-3


def test_lattice_max_call_single_date_is_the_integral():
    S0, sig = [100.0, 90.0], [0.2, 0.3]
    want = max_call_independent(S0, sig, 0.05, 0.02, 1.0, 100.0)
    v = oracle.lsm_lattice(S0, sig, 0.05, 0.02, 1.0, MAXC, 100.0, 1, 400)
    assert abs(v - want) < 1e-4


@pytest.mark.parametrize("d", [1, 2])
def test_lattice_call_without_dividends_is_never_exercised_early(d):
    # e^{-rh} E[(S' - K)+] >= (S - e^{-rh} K)+ >= (S - K)+ node by node when
    # q = 0 and r >= 0, so every exercise date leaves the value unchanged.
    S0, sig = [100.0, 95.0][:d], [0.2, 0.3][:d]
    kind = CALL if d == 1 else MAXC
    nt = 400 if d == 1 else 120
    euro = oracle.lsm_lattice(S0, sig, 0.05, 0.0, 1.0, kind, 100.0, 1, nt)
    berm = oracle.lsm_lattice(S0, sig, 0.05, 0.0, 1.0, kind, 100.0, 4, nt // 4)
    assert berm == pytest.approx(euro, rel=1e-12)


def test_lattice_put_value_rises_with_exercise_dates():
    # Same 400-step tree; more dates = a larger set of stopping rules.
    vals = [oracle.lsm_lattice([100.0], [0.2], 0.05, 0.0, 1.0, PUT, 100.0, M, 400 // M)
            for M in (1, 2, 4, 8, 16)]
    assert all(b > a + 1e-3 for a, b in zip(vals, vals[1:]))
    # A 400-step tree is within about 2/400 of Black-Scholes at the money.
    assert vals[0] == pytest.approx(bs_put_div(100.0, 100.0, 0.05, 0.0, 0.2, 1.0), abs=1e-2)


def test_lattice_reproduces_the_papers_max_call_value():
    g = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))["lsm_max_call"]
    v = oracle.lsm_lattice(g["S0"], g["sigma"], g["r"], g["q"], g["T"], MAXC, g["K"],
                           g["n_dates"], 50)
    assert abs(v - g["price"]) < 0.005


# ---- the estimator -----------------------------------------------------------
@pytest.mark.parametrize("kind,d,degree", [(MAXC, 2, 2), (PUT, 1, 3), (MAXC, 3, 1)])
def test_each_regression_is_least_squares_on_the_in_the_money_paths(kind, d, degree):
    S0 = np.array([100.0, 105.0, 95.0][:d])
    sig = np.array([0.2, 0.25, 0.3][:d])
    corr = np.full((d, d), 0.3) + 0.7 * np.eye(d)
    L = np.linalg.cholesky(corr)
    r, q, T, K, M = 0.05, 0.08, 2.0, 100.0, 5
    o = oracle.lsm(S0, sig, L, r, q, T, kind, K, M, 2, degree, 4096, SEED, want_paths=True)
    y, beta = o["y"], o["beta"]
    assert o["n_features"] == _feat(y[:, 0], y[:, 0, 0], degree, kind).shape[1]
    # Rebuild the cash flows date by date from the oracle's own betas.
    c = math.exp(-r * T) * K * _payoff(kind, y[:, M - 1])
    for j in range(M - 1, 0, -1):
        f = _payoff(kind, y[:, j - 1])
        itm = f > 0
        X = _feat(y[itm, j - 1], f[itm], degree, kind)
        want, *_ = np.linalg.lstsq(X, c[itm], rcond=None)
        assert np.allclose(beta[j - 1], want, rtol=1e-7, atol=1e-7 * np.abs(want).max())
        assert o["n_itm"][j - 1] == itm.sum()
        h = X @ beta[j - 1]
        dj = math.exp(-r * T * j / M)
        ex = dj * K * f[itm] >= h
        cj = c[itm]
        cj[ex] = dj * K * f[itm][ex]
        c[itm] = cj
    assert np.allclose(o["C"], c, rtol=1e-12, atol=1e-12)
    assert o["price"] == pytest.approx(c.mean(), rel=1e-12)
    assert np.isnan(beta[M - 1]).all()


def test_estimator_converges_to_the_lattice_for_the_max_call():
    g = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))["lsm_max_call"]
    true = oracle.lsm_lattice(g["S0"], g["sigma"], g["r"], g["q"], g["T"], MAXC, g["K"],
                              g["n_dates"], 50)
    args = (g["S0"], g["sigma"], np.eye(2), g["r"], g["q"], g["T"], MAXC, g["K"], g["n_dates"],
            1, 2)
    o = oracle.lsm(*args, 1 << 16, SEED)
    oos = oracle.lsm_oos(*args, o["beta"], 1 << 16, SEED, tag=7)
    # Regression bias is below 1% with these features; the out-of-sample rule
    # is a stopping rule, so its expectation is at most the true value.
    assert abs(o["price"] - true) < 3 * o["std_err"] + 0.01 * true
    assert oos["price"] < true + 3 * oos["std_err"]
    assert oos["price"] > true - 3 * oos["std_err"] - 0.01 * true
    # Early exercise is worth something here (dividend yield 0.1).
    assert o["price"] > o["european"] + 10 * o["std_err"]


def test_estimator_converges_to_the_lattice_for_the_put():
    true = oracle.lsm_lattice([100.0], [0.2], 0.05, 0.0, 1.0, PUT, 100.0, 10, 200)
    args = ([100.0], [0.2], np.eye(1), 0.05, 0.0, 1.0, PUT, 100.0, 10, 5, 3)
    o = oracle.lsm(*args, 1 << 16, SEED)
    oos = oracle.lsm_oos(*args, o["beta"], 1 << 16, SEED, tag=7)
    assert abs(o["price"] - true) < 3 * o["std_err"] + 0.01 * true
    assert oos["price"] < true + 3 * oos["std_err"]
    assert oos["price"] > true - 3 * oos["std_err"] - 0.01 * true


def test_call_without_dividends_matches_black_scholes():
    o = oracle.lsm([100.0], [0.2], np.eye(1), 0.05, 0.0, 1.0, CALL, 100.0, 8, 2, 2, 1 << 15, SEED)
    want = bs_call_div(100.0, 100.0, 0.05, 0.0, 0.2, 1.0)
    assert abs(o["european"] - want) < 4 * o["european_se"]
    # Early exercise is never optimal; the fitted rule stays close to never
    # exercising (in-sample it may gain or lose a little on the same paths).
    assert abs(o["price"] - o["european"]) < 0.5 * o["std_err"]


def test_single_date_is_the_european_estimate():
    o = oracle.lsm([100.0, 90.0], [0.2, 0.3], np.eye(2), 0.05, 0.1, 1.0, MAXC, 100.0, 1, 16, 2,
                   4096, SEED)
    assert o["price"] == o["european"]
    assert np.isnan(o["beta"]).all()
    assert set(np.unique(o["ex"])) <= {0, 1}


def test_out_of_the_money_everywhere_prices_zero():
    o = oracle.lsm([100.0], [0.2], np.eye(1), 0.05, 0.0, 1.0, CALL, 1e6, 6, 1, 2, 2048, SEED)
    assert o["price"] == 0.0 and o["std_err"] == 0.0
    assert np.isnan(o["beta"]).all() and (o["n_itm"] == 0).all() and (o["ex"] == 0).all()


def test_fewer_in_the_money_paths_than_features_skips_the_date():
    # 16 paths: some dates have fewer than 7 in-the-money paths.
    o = oracle.lsm([100.0, 100.0], [0.2, 0.2], np.eye(2), 0.05, 0.1, 3.0, MAXC, 125.0, 9, 1, 2,
                   16, SEED)
    skipped = o["n_itm"][:-1] < o["n_features"]
    assert skipped.any()
    assert np.isnan(o["beta"][:-1][skipped]).all()
    assert not np.isin(np.nonzero(skipped)[0] + 1, o["ex"]).any()


def test_out_of_sample_with_inactive_rule_is_the_european_payoff():
    args = ([100.0, 90.0], [0.2, 0.3], np.eye(2), 0.05, 0.1, 1.0, MAXC, 100.0, 4, 2, 2)
    nf = oracle.lsm_n_features(2, 2, MAXC)
    nan_beta = np.full((4, nf), np.nan)
    oos = oracle.lsm_oos(*args, nan_beta, 4096, SEED, tag=7)
    same = oracle.lsm(*args, 4096, SEED, tag=7)
    assert oos["price"] == pytest.approx(same["european"], rel=1e-14)


def test_feature_counts():
    # 1 + d + d(d+1)/2 (+ d(d+1)(d+2)/6) monomials, + f/K for the max-call.
    assert oracle.lsm_n_features(1, 3, PUT) == 4
    assert oracle.lsm_n_features(2, 2, MAXC) == 7
    assert oracle.lsm_n_features(2, 2, PUT) == 6
    assert oracle.lsm_n_features(2, 3, MAXC) == 11
    assert oracle.lsm_n_features(3, 2, MAXC) == 11
    assert oracle.lsm_n_features(4, 1, CALL) == 5
