"""GPU parity of the portfolio risk path (Sec. VI-B.1): the basket kernel's
per-path horizon P&L of a call portfolio under real-world drifts against
the FP64 oracle, the device order statistic and tail sum against the
definitions applied to the device's own path values (bit-exact rank,
FP64-rounding tail mean), VaR and CVaR against the oracle's on the same
paths within the largest per-path difference, full-size sampled paths,
determinism and argument errors."""
import math

import numpy as np
import pytest

import oracle
import paper_1906_02818_amd as mc
import synth

pytestmark = pytest.mark.gpu
SEED = synth.SEED
M5 = [0.9, 0.95, 1.0, 1.05, 1.1]
Q5 = [1.0, -2.0, 1.5, -1.0, 0.5]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mc.mc_create(0)
    yield c
    c.close()


def market(d):
    sigma, corr, _ = synth.basket_market(d)
    S0 = np.linspace(60.0, 140.0, d)
    mu = np.linspace(-0.02, 0.10, d)
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=S0, r=0.03, T=1.0, sigma=sigma, corr=corr)
    return model, S0, sigma, corr, oracle.cholesky(corr), mu


def check_selection(res, pnl, alpha):
    """Rank and tail of the device result against its own path values."""
    x = np.sort(pnl)
    N = x.size
    k = int(math.floor(N * (1.0 - alpha))) + 1
    assert res["k"] == k
    assert res["quantile_pnl"] == x[k - 1] and res["var"] == -x[k - 1]
    tail = x[x < x[k - 1]]
    assert res["n_tail"] == tail.size
    np.testing.assert_allclose(res["cvar"], -tail.mean(), rtol=1e-12)


@pytest.mark.parametrize("d,N,n,prec,offset,alpha", [
    (16, 4096, 8, mc.MC_FP32, 0, 0.95),
    (32, 1000, 5, mc.MC_FP32, 77, 0.99),
    (48, 3000, 3, mc.MC_BF16_GEMM, 0, 0.9),
    (16, 2500, 12, mc.MC_FP16_GEMM, (1 << 32) - 40, 0.95),
])
def test_risk_parity_small(ctx, d, N, n, prec, offset, alpha):
    say("risk", d, N, n, prec, offset, alpha)
    model, S0, sigma, corr, L, mu = market(d)
    r = mc.mc_risk(ctx, model, M5, Q5, alpha, N, n, SEED, mu=mu,
                   opts=mc.Options(prec=prec, path_offset=offset, path_values=True))
    o = oracle.portfolio_pnl(S0, sigma, mu, L, M5, Q5, 0.03, 1.0, n, N, SEED, path0=offset)
    gross = float(np.sum(S0) * np.sum(np.abs(Q5)))
    np.testing.assert_allclose(r["premium"],
                               oracle.portfolio_premium(S0, sigma, M5, Q5, 0.03, 1.0), rtol=1e-12)
    pnl = r["pnl"]
    assert r["n_paths"] == N
    diff = np.abs(pnl - o)
    if prec == mc.MC_FP32:
        assert diff.max() < 2e-6 * gross, diff.max()
    else:
        # Reduced-precision increments: per-path error of the product rounding.
        assert diff.max() < 2e-3 * gross, diff.max()
    check_selection(r, pnl, alpha)
    ov, oc, ok, _ = oracle.var_cvar(o, alpha)
    assert ok == r["k"]
    # An order statistic moves by at most the largest per-path change; so
    # does the mean of the tail set, up to a boundary swap.
    assert abs(r["var"] - ov) <= diff.max() * (1 + 1e-9) + 1e-12
    assert abs(r["cvar"] - oc) <= 2 * diff.max() + 1e-9
    np.testing.assert_allclose(r["pnl_mean"], pnl.mean(), rtol=1e-10, atol=1e-9 * gross)


def test_risk_full_size_sampled(ctx):
    # The benchmarked shape: d = 256, 2^20 paths, 100 steps; selection exact
    # over all paths, P&L against the oracle on sampled paths.
    say("risk full size")
    c = synth.BASKET
    d, N, n = c["d"], 1 << 20, c["n_steps"]
    model, S0, sigma, corr, L, mu = market(d)
    r = mc.mc_risk(ctx, model, M5, Q5, 0.95, N, n, SEED, mu=mu,
                   opts=mc.Options(prec=mc.MC_FP32, path_values=True))
    pnl = r["pnl"]
    check_selection(r, pnl, 0.95)
    gross = float(np.sum(S0) * np.sum(np.abs(Q5)))
    for p0 in (0, 123457, N - 32):
        o = oracle.portfolio_pnl(S0, sigma, mu, L, M5, Q5, 0.03, 1.0, n, 32, SEED, path0=p0)
        assert np.abs(pnl[p0:p0 + 32] - o).max() < 2e-6 * gross


def test_risk_deterministic(ctx):
    model, S0, sigma, corr, L, mu = market(32)
    a = mc.mc_risk(ctx, model, M5, Q5, 0.95, 20000, 6, SEED, mu=mu)
    b = mc.mc_risk(ctx, model, M5, Q5, 0.95, 20000, 6, SEED, mu=mu)
    assert a["var"] == b["var"] and a["cvar"] == b["cvar"] and a["pnl_mean"] == b["pnl_mean"]


@pytest.mark.parametrize("kw,status", [
    (dict(alpha=1.0), mc.MC_ERR_INVALID_ARG),
    (dict(alpha=0.0), mc.MC_ERR_INVALID_ARG),
    (dict(N=19, alpha=0.95), mc.MC_ERR_INVALID_ARG),          # k = 1: empty tail
    (dict(m=[-0.5], q=[1.0]), mc.MC_ERR_INVALID_ARG),
    (dict(m=[1.0], q=[float("nan")]), mc.MC_ERR_INVALID_ARG),
    (dict(prec=mc.MC_BF16X2_GEMM), mc.MC_ERR_UNSUPPORTED),
    (dict(prec=mc.MC_FP64), mc.MC_ERR_UNSUPPORTED),
    (dict(mu_bad=True), mc.MC_ERR_INVALID_ARG),
])
def test_risk_argument_errors(ctx, kw, status):
    model, S0, sigma, corr, L, mu = market(16)
    if kw.get("mu_bad"):
        mu = mu.copy()
        mu[3] = np.inf
    with pytest.raises(mc.McError) as e:
        mc.mc_risk(ctx, model, kw.get("m", M5), kw.get("q", Q5), kw.get("alpha", 0.95),
                   kw.get("N", 1000), 4, SEED, mu=mu,
                   opts=mc.Options(prec=kw.get("prec", mc.MC_FP32)))
    assert e.value.status == status


def test_risk_needs_the_basket_model(ctx):
    gbm = mc.Model(kind=mc.MC_GBM, S0=100.0, r=0.03, T=1.0, sigma=0.2)
    with pytest.raises(mc.McError) as e:
        mc.mc_risk(ctx, gbm, [1.0], [1.0], 0.95, 1000, 4, SEED)
    assert e.value.status == mc.MC_ERR_UNSUPPORTED
