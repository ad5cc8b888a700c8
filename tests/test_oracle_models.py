"""Pins of the oracle's path simulators against what the mathematics fixes:
closed forms, exact moments, invariants, finite differences and special
cases that reduce to a textbook routine. Each test is chosen so that a
plausible slip (a dropped drift term, a wrong sign, a swapped normal, a
transposed factor) fails it.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from closed_forms import (arith_asian2_call, bs_call, bs_delta, bs_vega, geo_asian_call, up_out_call,
                          bgk_discrete_up_out_call, heston_call, geo_basket_call)

HERE = os.path.dirname(os.path.abspath(__file__))


def within(est, ref, k=4.0, extra=0.0):
    return abs(est["price"] - ref) <= k * est["std_err"] + extra


# --- GBM (Sec. II-A.1 scheme, Sec. VI-A.1 workloads) ----------------------
def test_paper_vanilla_call_value():
    g = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))["vanilla_call"]
    ref = bs_call(g["S0"], g["K"], g["r"], g["sigma"], g["T"])
    assert abs(ref - g["price"]) < 1e-10
    o = oracle.gbm(g["S0"], g["r"], g["sigma"], g["T"], g["K"], 1e30, 25, 1 << 17, 1234)
    assert within(oracle.estimate(o[:, 0]), g["price"])


def test_gbm_european_price_delta_vega_closed_form():
    c = synth.EURO
    o = oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], 1e30, c["n_steps"],
                   c["n_paths"], synth.SEED)
    args = (c["S0"], c["K"], c["r"], c["sigma"], c["T"])
    assert within(oracle.estimate(o[:, 0]), bs_call(*args))
    assert within(oracle.estimate(o[:, 4]), bs_delta(*args))
    assert within(oracle.estimate(o[:, 5]), bs_vega(*args))
    # Discounted terminal price is a martingale under log-Euler.
    assert within(oracle.estimate(o[:, 8]), c["S0"])
    # A closed form for the wrong rate or vol would be far away.
    assert not within(oracle.estimate(o[:, 0]), bs_call(c["S0"], c["K"], 0.0, c["sigma"], 1.0))


def test_geometric_asian_closed_form_and_ordering():
    c = synth.ASIAN_BARRIER
    o = oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], c["B"], c["n_steps"],
                   1 << 16, synth.SEED)
    ref = geo_asian_call(c["S0"], c["K"], c["r"], c["sigma"], c["T"], c["n_steps"])
    assert abs(ref - 6.120881255555376) < 1e-9
    assert within(oracle.estimate(o[:, 2]), ref)
    # Arithmetic mean >= geometric mean path by path.
    assert np.all(o[:, 1] >= o[:, 2] - 1e-12)
    # Asian delta is the average of S_i/S0 on the in-the-money paths.
    d = oracle.estimate(o[:, 6])["price"]
    assert 0.3 < d < 0.8


def test_barrier_special_cases_and_bounds():
    c = synth.ASIAN_BARRIER
    o = oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], 1e30, 64, 4096, 5)
    assert np.array_equal(o[:, 3], o[:, 0])           # barrier at infinity = European
    assert np.array_equal(o[:, 9], o[:, 0])
    o = oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], c["B"], c["n_steps"],
                   1 << 16, synth.SEED)
    uo = oracle.estimate(o[:, 3])
    cont = up_out_call(c["S0"], c["K"], c["B"], c["r"], c["sigma"], c["T"])
    bgk = bgk_discrete_up_out_call(c["S0"], c["K"], c["B"], c["r"], c["sigma"], c["T"],
                                   c["n_steps"])
    assert abs(cont - 2.1766071418) < 1e-9
    assert within(uo, bgk, extra=0.01)
    assert uo["price"] > cont + 2 * uo["std_err"]     # discrete monitoring knocks out less
    assert np.all(o[:, 3] <= o[:, 0])


def test_brownian_bridge_barrier_matches_continuous_closed_form():
    # With the bridge maximum drawn between grid points the log-Euler GBM
    # barrier is exact in law: it must match the continuous formula at any n.
    c = synth.ASIAN_BARRIER
    for n in (8, 64):
        o = oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], c["B"], n, 1 << 17,
                       synth.SEED)
        cont = up_out_call(c["S0"], c["K"], c["B"], c["r"], c["sigma"], c["T"])
        assert within(oracle.estimate(o[:, 9]), cont)
        assert np.all(o[:, 9] <= o[:, 3])


def test_euler_on_S_moments_and_first_order_weak_error():
    # Euler on S: E[S_n] = S0 (1 + r dt)^n and
    # E[S_n^2] = S0^2 ((1 + r dt)^2 + sigma^2 dt)^n exactly.
    S0, r, sig, T, K = 100.0, 0.05, 0.2, 1.0, 100.0
    disc = math.exp(-r * T)
    for n in (2, 16):
        dt = T / n
        o = oracle.gbm(S0, r, sig, T, K, 1e30, n, 1 << 18, 3, scheme=1)
        assert within(oracle.estimate(o[:, 8]), disc * S0 * (1 + r * dt) ** n)
        m2 = disc ** 2 * S0 ** 2 * ((1 + r * dt) ** 2 + sig * sig * dt) ** n
        assert within(oracle.estimate(o[:, 8] ** 2), m2)
    # n = 2 is far from the continuous second moment (bias of order dt).
    cont2 = disc ** 2 * S0 ** 2 * math.exp((2 * r + sig * sig) * T)
    o = oracle.gbm(S0, r, sig, T, K, 1e30, 2, 1 << 18, 3, scheme=1)
    assert not within(oracle.estimate(o[:, 8] ** 2), cont2)
    # Talay-Tubaro (Sec. V-B): the weak error of the call is O(1/n), so with
    # coupled levels E[P_n - P_2n] / E[P_2n - P_4n] is close to 2 (an
    # O(sqrt(dt)) error would give sqrt(2), an O(dt^2) one 4). The paper's
    # vanilla call (K = 120) has the coupled differences with the best
    # signal to noise: at 2^20 paths the ratio's standard error is about
    # 0.05 at n = 16 and 0.08 at n = 32.
    Kp = 120.0
    for n in (16, 32):
        f4 = oracle.gbm(S0, r, sig, T, Kp, 1e30, 4 * n, 1 << 20, 7, scheme=1, coarsen=1)[:, 0]
        f2 = oracle.gbm(S0, r, sig, T, Kp, 1e30, 2 * n, 1 << 20, 7, scheme=1, coarsen=2)[:, 0]
        f1 = oracle.gbm(S0, r, sig, T, Kp, 1e30, n, 1 << 20, 7, scheme=1, coarsen=4)[:, 0]
        d1, d2 = oracle.estimate(f1 - f2), oracle.estimate(f2 - f4)
        assert d2["price"] < -20 * d2["std_err"]   # Euler on S biases the call down
        ratio = d1["price"] / d2["price"]
        assert 1.7 < ratio < 2.4, (n, ratio)
    # The log-Euler scheme has no bias for the European call at any n.
    for n in (2, 8):
        o = oracle.gbm(S0, r, sig, T, K, 1e30, n, 1 << 18, 9)
        assert within(oracle.estimate(o[:, 0]), bs_call(S0, K, r, sig, T))


def test_gbm_pathwise_tangents_match_common_random_number_fd():
    S0, r, sig, T, K = 100.0, 0.03, 0.25, 1.0, 100.0
    n, N = 32, 1 << 14
    base = oracle.gbm(S0, r, sig, T, K, 1e30, n, N, 21)
    for scheme in (0, 1):
        base = oracle.gbm(S0, r, sig, T, K, 1e30, n, N, 21, scheme=scheme)
        h = 1e-3 * S0
        up = oracle.gbm(S0 + h, r, sig, T, K, 1e30, n, N, 21, scheme=scheme)
        dn = oracle.gbm(S0 - h, r, sig, T, K, 1e30, n, N, 21, scheme=scheme)
        for ch, dch in ((0, 4), (1, 6)):
            fd = (up[:, ch] - dn[:, ch]) / (2 * h)
            diff = oracle.estimate(base[:, dch] - fd)
            assert abs(diff["price"]) < 4 * diff["std_err"] + 1e-6
        h = 1e-3 * sig
        up = oracle.gbm(S0, r, sig + h, T, K, 1e30, n, N, 21, scheme=scheme)
        dn = oracle.gbm(S0, r, sig - h, T, K, 1e30, n, N, 21, scheme=scheme)
        for ch, dch in ((0, 5), (1, 7)):
            fd = (up[:, ch] - dn[:, ch]) / (2 * h)
            diff = oracle.estimate(base[:, dch] - fd)
            assert abs(diff["price"]) < 4 * diff["std_err"] + 1e-4


def test_rmse_decays_as_inverse_sqrt_n():
    # Sec. VI-D: Monte Carlo RMSE falls as N^{-1/2}. Log-Euler is exact in
    # law, so the error against Black-Scholes is pure sampling error. 128
    # seeds at six sizes from 2^6 to 2^16 put the fitted slope's standard
    # error near 0.012, so the window is about four of them.
    S0, r, sig, T, K = 100.0, 0.05, 0.2, 1.0, 100.0
    ref = bs_call(S0, K, r, sig, T)
    Ns = [1 << k for k in range(6, 17, 2)]
    rmse = []
    for N in Ns:
        errs = [oracle.estimate(oracle.gbm(S0, r, sig, T, K, 1e30, 1, N, 1000 + s)[:, 0])["price"]
                - ref for s in range(128)]
        rmse.append(math.sqrt(np.mean(np.square(errs))))
    slope = np.polyfit(np.log(Ns), np.log(rmse), 1)[0]
    assert -0.55 < slope < -0.45, slope


# --- Heston ---------------------------------------------------------------
H = {k: synth.HESTON[k] for k in ("S0", "v0", "kappa", "theta", "xi", "rho", "r", "T", "K")}


def _heston(n, N, seed, **over):
    p = dict(H)
    p.update(over)
    return oracle.heston(p["S0"], p["v0"], p["kappa"], p["theta"], p["xi"], p["rho"], p["r"],
                         p["T"], p["K"], n, N, seed)


def _hcf(**over):
    p = dict(H)
    p.update(over)
    return heston_call(p["S0"], p["v0"], p["kappa"], p["theta"], p["xi"], p["rho"], p["r"],
                       p["T"], p["K"])


def test_heston_european_matches_characteristic_function():
    ref = _hcf()
    assert abs(ref - 8.3357914938) < 1e-8
    o = _heston(64, 1 << 17, synth.SEED)
    assert within(oracle.estimate(o[:, 0]), ref, extra=0.01)
    # Discounted S is a martingale under full-truncation log-Euler.
    assert within(oracle.estimate(o[:, 6]), H["S0"])
    # The sign of rho shows in the skew: out of the money (K = 125) the
    # rho = +0.7 and rho = -0.7 prices are far apart, and each matches its CF.
    for rho in (-0.7, 0.7):
        e = oracle.estimate(_heston(64, 1 << 17, synth.SEED, rho=rho, K=125.0)[:, 0])
        assert within(e, _hcf(rho=rho, K=125.0), extra=0.01)
    gap = _hcf(rho=0.7, K=125.0) - _hcf(rho=-0.7, K=125.0)
    assert gap > 20 * e["std_err"]


def test_heston_discretisation_bias_shrinks():
    ref = _hcf()
    prev = None
    for n in (2, 4, 8):
        b = oracle.estimate(_heston(n, 1 << 17, 77)[:, 0])["price"] - ref
        if prev is not None:
            assert b < prev
        prev = b
    assert prev > 0


def test_heston_greeks_match_cf_and_fd():
    o = _heston(64, 1 << 17, synth.SEED)
    h = 1e-4
    cf_delta = (_hcf(S0=H["S0"] * (1 + h)) - _hcf(S0=H["S0"] * (1 - h))) / (2 * h * H["S0"])
    cf_dv0 = (_hcf(v0=H["v0"] * (1 + h)) - _hcf(v0=H["v0"] * (1 - h))) / (2 * h * H["v0"])
    assert abs(cf_delta - 0.670054) < 2e-6
    assert abs(cf_dv0 - 40.4108) < 2e-3
    assert within(oracle.estimate(o[:, 2]), cf_delta, extra=1e-3)
    assert within(oracle.estimate(o[:, 3]), cf_dv0, k=5.0, extra=0.3)
    # Pathwise tangents of the Asian vs central FD on common random numbers.
    N, n = 1 << 13, 32
    base = _heston(n, N, 5)
    for key, ch, col in (("S0", 1, 4), ("v0", 1, 5)):
        hh = 1e-3 * H[key]
        up = _heston(n, N, 5, **{key: H[key] + hh})
        dn = _heston(n, N, 5, **{key: H[key] - hh})
        fd = (up[:, ch] - dn[:, ch]) / (2 * hh)
        diff = oracle.estimate(base[:, col] - fd)
        scale = abs(oracle.estimate(base[:, col])["price"])
        assert abs(diff["price"]) < 4 * diff["std_err"] + 1e-3 * scale


# --- Basket (Sec. II-A.2, Sec. VI-A.2) --------------------------------------
def test_cholesky_reconstructs_and_matches_numpy():
    sigma, corr, lam = synth.basket_market(64)
    assert lam >= 0.05
    L = oracle.cholesky(corr)
    assert np.max(np.abs(L @ L.T - corr)) < 1e-12
    assert np.max(np.abs(L - np.linalg.cholesky(corr))) < 1e-12
    assert np.all(np.triu(L, 1) == 0.0)
    bad = corr.copy()
    bad[0, 1] = bad[1, 0] = 1.5
    assert oracle.cholesky(bad) is None


def test_basket_one_asset_reduces_to_gbm():
    o = oracle.basket([100.0], [0.2], np.ones((1, 1)), [1.0], 0.05, 1.0, 100.0, 16, 2048, 3)
    g = oracle.gbm(100.0, 0.05, 0.2, 1.0, 100.0, 1e30, 16, 2048, 3)
    np.testing.assert_allclose(o[:, 0], g[:, 0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(o[:, 2], g[:, 4], rtol=1e-12, atol=1e-12)


def test_geometric_basket_closed_form():
    d = 16
    sigma, corr, _ = synth.basket_market(d)
    L = oracle.cholesky(corr)
    S0 = np.full(d, 100.0)
    w = np.full(d, 1.0 / d)
    o = oracle.basket(S0, sigma, L, w, 0.05, 1.0, 100.0, 10, 1 << 16, synth.SEED)
    ref = geo_basket_call(S0, sigma, corr, w, 0.05, 1.0, 100.0)
    assert within(oracle.estimate(o[:, 1]), ref)
    # Using L^T instead of L would give a different covariance.
    wrong = geo_basket_call(S0, sigma, (L.T @ L), w, 0.05, 1.0, 100.0)
    assert abs(wrong - ref) > 8 * oracle.estimate(o[:, 1])["std_err"]
    assert np.all(o[:, 0] >= o[:, 1] - 1e-12)      # arithmetic >= geometric


# --- Learned control variate ---------------------------------------------
def test_hedge_pnl_has_zero_mean_for_random_weights():
    rng = np.random.default_rng(3)
    theta = rng.normal(0.0, 0.5, oracle.MLP_NPARAM)
    o = oracle.heston_cv(H, 16, theta, 1 << 15, synth.SEED)
    assert within(oracle.estimate(o[:, 1]), 0.0)
    plain = oracle.estimate(o[:, 0])
    cv = oracle.estimate(o[:, 2])
    assert abs(cv["price"] - plain["price"]) < 3 * math.hypot(cv["std_err"], plain["std_err"])
    o4 = oracle.heston_cv(H, 16, theta, 1 << 15, synth.SEED, m_every=4)
    assert within(oracle.estimate(o4[:, 1]), 0.0)
    np.testing.assert_array_equal(o4[:, 0], o[:, 0])
    # Payoff channel equals the plain Heston Asian channel path by path.
    hp = _heston(16, 1 << 10, synth.SEED)
    np.testing.assert_allclose(o[: 1 << 10, 0], hp[:, 1], rtol=1e-13, atol=1e-13)


def test_mlp_backprop_matches_finite_differences():
    rng = np.random.default_rng(5)
    theta = synth.glorot_mlp() + rng.normal(0, 0.05, oracle.MLP_NPARAM)
    loss, grad = oracle.cv_loss_grad(H, 6, theta, 48, synth.SEED, m_every=2)
    idx = np.concatenate([rng.choice(256, 6, replace=False),
                          256 + rng.choice(64, 3, replace=False),
                          320 + rng.choice(4096, 8, replace=False),
                          4416 + rng.choice(64, 3, replace=False),
                          4480 + rng.choice(64, 4, replace=False), [4544]])
    for i in idx:
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = oracle.cv_loss_grad(H, 6, tp, 48, synth.SEED, m_every=2, want_grad=False)
        lm, _ = oracle.cv_loss_grad(H, 6, tm, 48, synth.SEED, m_every=2, want_grad=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (i, fd, grad[i])
    # The b3 (constant hedge) gradient is -(2/B) sum (Y - Ybar) * sum dSt.
    assert loss > 0


def test_bf16_rounding_matches_torch():
    # Round to nearest, ties to even, on the top 16 bits of the FP32 value:
    # random magnitudes, exact ties with even and odd kept bits, subnormals.
    import torch
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1, 500) * 10.0 ** rng.integers(
        -40, 38, 500), [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40, -1e-41]])
    ties = np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x00018000, 0x40490FDB],
                    np.uint32).view(np.float32).astype(np.float64)
    x = np.concatenate([x, ties])
    want = torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).double()
    got = np.array([oracle.bf16_round(v) for v in x])
    np.testing.assert_array_equal(got, want.numpy())


def test_mlp_bf16_operands_match_rounded_forward():
    # The bfloat16 network: operands of both matrix products rounded to
    # bfloat16, everything else in double precision.
    import torch

    def bf(a):
        return torch.tensor(np.asarray(a, np.float64)).to(torch.float32).to(
            torch.bfloat16).double().numpy()
    rng = np.random.default_rng(12)
    theta = synth.glorot_mlp() + rng.normal(0, 0.2, oracle.MLP_NPARAM)
    phi = rng.normal(0, 0.7, (300, 4))
    W1, b1 = theta[:256].reshape(64, 4), theta[256:320]
    W2, b2 = theta[320:4416].reshape(64, 64), theta[4416:4480]
    W3, b3 = theta[4480:4544], theta[4544]
    h1 = np.tanh(bf(phi) @ bf(W1).T + bf(b1))
    h2 = np.tanh(bf(h1) @ bf(W2).T + b2)
    want = h2 @ W3 + b3
    got = oracle.mlp_eval(theta, phi, bf16=True)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    exact = np.tanh(np.tanh(phi @ W1.T + b1) @ W2.T + b2) @ W3 + b3
    np.testing.assert_allclose(oracle.mlp_eval(theta, phi), exact, rtol=1e-12, atol=1e-12)
    d = np.abs(got - exact)
    assert 0 < d.max() < 3e-2 * np.abs(exact).max()


def test_adam_matches_definition_on_a_quadratic():
    # Adam's first step moves every coordinate by lr * sign(grad).
    th = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    t1, m, v = oracle.adam_step(th, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    np.testing.assert_allclose(t1, th - 0.1 * np.sign(g), rtol=1e-6)
    # Minimises a convex quadratic.
    x, m, v = np.array([5.0, -3.0]), np.zeros(2), np.zeros(2)
    for t in range(1, 3001):
        x, m, v = oracle.adam_step(x, 2 * x, m, v, t, lr=0.05)
    assert np.max(np.abs(x)) < 1e-2


def test_arithmetic_average_mean_is_exact_at_zero_strike():
    # With K = 0 the Asian payoff is e^{-rT} A, and E[A] = (S0/n) sum_i e^{r t_i}
    # for any martingale-preserving scheme (log-Euler GBM and full-truncation
    # log-Euler Heston). Including S0 in the average, or dividing by n+1,
    # would move it by several standard errors.
    S0, r, sig, T, n = 100.0, 0.03, 0.25, 1.0, 4
    exact = math.exp(-r * T) * S0 / n * sum(math.exp(r * i * T / n) for i in range(1, n + 1))
    wrong = math.exp(-r * T) * S0 / (n + 1) * sum(math.exp(r * i * T / n) for i in range(0, n + 1))
    o = oracle.gbm(S0, r, sig, T, 0.0, 1e30, n, 1 << 20, 17)
    e = oracle.estimate(o[:, 1])
    assert within(e, exact) and not within(e, wrong)
    oh = _heston(n, 1 << 20, 17, K=0.0, r=r)
    e = oracle.estimate(oh[:, 1])
    assert within(e, exact) and not within(e, wrong)


@pytest.mark.parametrize("K", [95.0, 101.0, 120.0])
def test_asian_price_at_zero_volatility_is_the_deterministic_payoff(K):
    # sigma = 0: every path is S_{t_i} = S0 e^{r t_i}, so the Asian channel is
    # e^{-rT} (A - K)^+ with A the mean of the n fixings, exactly, on every
    # path: this pins the strike, the positive part and the discounting of
    # the K > 0 payoff, which the K = 0 mean above cannot see.
    S0, r, T, n = 100.0, 0.03, 1.0, 12
    A = S0 / n * sum(math.exp(r * i * T / n) for i in range(1, n + 1))
    want = math.exp(-r * T) * max(A - K, 0.0)
    o = oracle.gbm(S0, r, 0.0, T, K, 1e30, n, 64, 17)
    # Absolute tolerance: A - K cancels, and the path's log-price carries the
    # rounding of n accumulated steps (~1e-14 of S0).
    np.testing.assert_allclose(o[:, 1], want, rtol=0, atol=1e-11)
    geo = math.exp(-r * T) * max(math.exp(sum(math.log(S0) + r * i * T / n
                                               for i in range(1, n + 1)) / n) - K, 0.0)
    np.testing.assert_allclose(o[:, 2], geo, rtol=0, atol=1e-11)


@pytest.mark.parametrize("K", [90.0, 100.0, 115.0])
def test_arithmetic_asian_two_fixings_semi_closed_form(K):
    # The arithmetic-Asian price at K > 0 with volatility on two fixings,
    # S(T/2) and S(T): against the semi-closed form (inner Black-Scholes
    # given S(T/2), outer quadrature), for GBM and for Heston without
    # vol-of-vol (v0 = theta: GBM with sigma = sqrt(theta), exact in law under
    # the log-Euler step). Averaging S0 in, a wrong divisor, shifted fixings
    # or a half-period discount would each move the price by many standard
    # errors; so would the European or the geometric Asian in its place.
    S0, r, T, th = H["S0"], H["r"], H["T"], 0.0625
    sig = math.sqrt(th)
    ref = arith_asian2_call(S0, K, r, sig, T)
    o = oracle.gbm(S0, r, sig, T, K, 1e30, 2, 1 << 20, 41)
    e = oracle.estimate(o[:, 1])
    assert within(e, ref)
    assert not within(e, bs_call(S0, K, r, sig, T))
    assert not within(e, geo_asian_call(S0, K, r, sig, T, 2))
    oh = _heston(2, 1 << 20, 43, xi=0.0, v0=th, theta=th, K=K)
    assert within(oracle.estimate(oh[:, 1]), ref)
    # One fixing: the Asian channel is the European call.
    o1 = oracle.gbm(S0, r, sig, T, K, 1e30, 1, 4096, 47)
    np.testing.assert_allclose(o1[:, 1], o1[:, 0], rtol=1e-14, atol=1e-13)


def test_heston_without_vol_of_vol_is_black_scholes():
    # xi = 0 and v0 = theta: the variance stays at theta on every path, so the
    # full-truncation scheme is log-Euler GBM with sigma = sqrt(theta), exact
    # in law: the European channel is Black-Scholes within Monte Carlo error,
    # and its pathwise delta is the Black-Scholes delta.
    th = 0.04
    o = _heston(32, 1 << 18, 29, xi=0.0, v0=th, theta=th, rho=-0.7)
    S0, K, r, T = H["S0"], H["K"], H["r"], H["T"]
    e = oracle.estimate(o[:, 0])
    assert within(e, bs_call(S0, K, r, math.sqrt(th), T), 4.0)
    d = oracle.estimate(o[:, 2])
    assert within(d, bs_delta(S0, K, r, math.sqrt(th), T), 4.0)


def test_gbm_payoff_only_mode_equals_all_channels():
    # The oracle's payoff-only GBM mode (used to time the CPU baseline on the
    # channels the benchmarked step computes) gives the same payoff channels
    # bit for bit and leaves the rest undefined.
    for scheme in (0, 1):
        a = oracle.gbm(100.0, 0.03, 0.25, 1.0, 100.0, 130.0, 37, 513, 5, scheme=scheme)
        b = oracle.gbm(100.0, 0.03, 0.25, 1.0, 100.0, 130.0, 37, 513, 5, scheme=scheme,
                       payoffs_only=True)
        cols = [0, 1, 2, 3, 8]
        assert np.array_equal(a[:, cols], b[:, cols])
        assert np.isnan(b[:, [4, 5, 6, 7, 9, 10, 11]]).all()
