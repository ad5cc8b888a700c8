"""GPU parity of randomised Sobol' quasi-Monte Carlo on the basket kernel
(Sec. IV-B, Sec. VI-D): per-path channels against the FP64 oracle on the
same shifted points (one and several steps, point offsets, FP16), replicate
estimates against the oracle's, the geometric-basket closed form with an
RMSE that falls faster than N^(-1/2), and argument errors (BF16 products,
whose bias exceeds the QMC standard error, are refused)."""
import math

import numpy as np
import pytest

import oracle
import paper_1906_02818_amd as mc
import synth
from closed_forms import geo_basket_call

pytestmark = pytest.mark.gpu
SEED = synth.SEED


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mc.mc_create(0)
    yield c
    c.close()


def market(d, r=0.05):
    sigma, corr, _ = synth.basket_market(d)
    S0 = np.full(d, 100.0)
    w = np.full(d, 1.0 / d)
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=S0, r=r, T=1.0, sigma=sigma, corr=corr)
    return model, S0, sigma, corr, oracle.cholesky(corr), w


@pytest.mark.parametrize("d,N,n,offset,prec", [(16, 4096, 1, 0, mc.MC_FP32),
                                               (32, 3000, 3, 1000, mc.MC_FP32),
                                               (16, 2048, 2, 0, mc.MC_FP16_GEMM)])
def test_qmc_paths_match_oracle(ctx, d, N, n, offset, prec):
    say("qmc paths", d, N, n, offset, prec)
    model, S0, sigma, corr, L, w = market(d)
    r = mc.mc_price_qmc(ctx, model, mc.Payoff(mc.MC_BASKET_CALL, 100.0), N, n, SEED, 1,
                        mc.Options(prec=prec, path_offset=offset, path_values=True))
    o = oracle.basket_qmc(S0, sigma, L, w, 0.05, 1.0, 100.0, n, N, SEED, 0, tag=6, path0=offset)
    pv = r["path_values"]
    if prec == mc.MC_FP32:
        np.testing.assert_allclose(pv[:, 0], o[:, 0], rtol=1e-4, atol=1e-4)
        np.testing.assert_allclose(pv[:, 1], o[:, 1], rtol=1e-4, atol=1e-4)
    else:
        # FP16 increments: per-path error of the 11-bit-mantissa rounding of
        # Z and L (largest for the extreme normals of boundary points).
        diff = np.abs(pv[:, 0] - o[:, 0])
        assert diff.max() < 2e-3 * o[:, 0].max()
        assert diff.mean() < 3e-4 * o[:, 0].mean()
    np.testing.assert_allclose(r["price"], pv[:, 0].mean(), rtol=1e-12)


@pytest.mark.parametrize("d,N,n,R,offset", [(16, 2048, 1, 6, 0), (48, 2000, 2, 3, 777)])
def test_qmc_replicates_match_oracle(ctx, d, N, n, R, offset):
    # All replicates run in one launch; the second case has a ragged last
    # block in every replicate, two asset blocks and a point offset.
    say("qmc replicates", d, N, n, R, offset)
    model, S0, sigma, corr, L, w = market(d)
    r = mc.mc_price_qmc(ctx, model, mc.Payoff(mc.MC_BASKET_CALL, 100.0), N, n, SEED, R,
                        mc.Options(path_offset=offset))
    for rep in range(R):
        o = oracle.basket_qmc(S0, sigma, L, w, 0.05, 1.0, 100.0, n, N, SEED, rep, tag=6,
                              path0=offset)
        assert abs(r["replicate_price"][rep] - o[:, 0].mean()) < 2e-5 * o[:, 0].mean()
        assert abs(r["replicate_geo"][rep] - o[:, 1].mean()) < 2e-5 * o[:, 1].mean()
    est = np.array(r["replicate_price"])
    np.testing.assert_allclose(r["price"], est.mean(), rtol=1e-14)
    np.testing.assert_allclose(r["std_err"], est.std(ddof=1) / math.sqrt(R), rtol=1e-10)


def test_qmc_benchmarked_launch_matches_oracle(ctx):
    # The launch the benchmark times: 16 digital shifts of 2^16 points of the
    # 16-asset basket in one step, all replicates in one launch; the oracle
    # prices every replicate in full.
    d, N, n, R = 16, 1 << 16, 1, 16
    say("qmc benchmarked launch", d, N, R)
    model, S0, sigma, corr, L, w = market(d)
    h = mc.mc_price_qmc(ctx, model, mc.Payoff(mc.MC_BASKET_CALL, 100.0), N, n, SEED, R,
                        mc.Options(prec=mc.MC_FP16_GEMM))
    ref = mc.mc_price_qmc(ctx, model, mc.Payoff(mc.MC_BASKET_CALL, 100.0), N, n, SEED, R)
    om = np.array([oracle.basket_qmc(S0, sigma, L, w, 0.05, 1.0, 100.0, n, N, SEED, rep,
                                      tag=6)[:, 0].mean() for rep in range(R)])
    g32 = np.array(ref["replicate_price"][:R])
    # The reduced-precision errors against FP64, in QMC standard errors: the
    # bench line for this workload runs FP32 products.
    se = ref["std_err"]
    say(f"  oracle {om.mean():.8f}, FP32 {ref['price']:.8f} +- {se:.2e}; max rel FP32 "
        f"{np.abs(g32 / om - 1).max():.2e}; FP16 {h['price']:.8f} "
        f"({(h['price'] - om.mean()) / se:+.2f} SE)")
    # FP32 products: each replicate within 2e-5 of the oracle, and the
    # estimate within 0.1 standard errors of the oracle's.
    assert np.abs(g32 / om - 1).max() < 2e-5
    assert abs(ref["price"] - om.mean()) < 0.1 * se
    # FP16 products (L' to 11 bits) stay within 0.1 standard errors. BF16 (8
    # bits) moved this 16-asset price by about 4 of them, so the entry point
    # refuses it.
    assert abs(h["price"] - om.mean()) < 0.1 * se
    with pytest.raises(mc.McError) as e:
        mc.mc_price_qmc(ctx, model, mc.Payoff(mc.MC_BASKET_CALL, 100.0), N, n, SEED, R,
                        mc.Options(prec=mc.MC_BF16_GEMM))
    assert e.value.status == mc.MC_ERR_UNSUPPORTED


def test_qmc_geometric_closed_form_and_rate(ctx):
    # Unbiased for the closed form; RMSE over replicates well below the Monte
    # Carlo standard error at every size and falling faster than N^(-1/2).
    say("qmc rate")
    d, R = 16, 16
    model, S0, sigma, corr, L, w = market(d)
    f = mc.Payoff(mc.MC_BASKET_CALL, 100.0)
    exact = geo_basket_call(S0, sigma, corr, w, 0.05, 1.0, 100.0)
    pv = mc.mc_price_qmc(ctx, model, f, 1 << 14, 1, SEED, 1,
                         mc.Options(path_values=True))["path_values"][:, 1]
    sd = pv.std()
    Ns = [1 << 10, 1 << 12, 1 << 14, 1 << 16]
    rmse = []
    for N in Ns:
        r = mc.mc_price_qmc(ctx, model, f, N, 1, SEED, R)
        est = np.array(r["replicate_geo"])
        rmse.append(math.sqrt(np.mean((est - exact) ** 2)))
        assert rmse[-1] < 0.3 * sd / math.sqrt(N), (N, rmse[-1], sd / math.sqrt(N))
    assert abs(r["geo_price"] - exact) < 4 * r["geo_std_err"] + 2e-5 * exact
    slope = np.polyfit(np.log(Ns), np.log(rmse), 1)[0]
    say("rmse", rmse, "slope", slope)
    assert slope < -0.55


@pytest.mark.parametrize("kw,status", [
    (dict(R=0), mc.MC_ERR_INVALID_ARG),
    (dict(R=65), mc.MC_ERR_INVALID_ARG),
    (dict(offset=(1 << 32) - 100), mc.MC_ERR_INVALID_ARG),
    (dict(n=4097), mc.MC_ERR_INVALID_ARG),
    (dict(R=2, pv=True), mc.MC_ERR_UNSUPPORTED),
    (dict(prec=mc.MC_BF16X2_GEMM), mc.MC_ERR_UNSUPPORTED),
    (dict(prec=mc.MC_BF16_GEMM), mc.MC_ERR_UNSUPPORTED),
    (dict(prec=mc.MC_BF16_GEMM, R=1, pv=True), mc.MC_ERR_UNSUPPORTED),
])
def test_qmc_argument_errors(ctx, kw, status):
    model, *_ = market(16)
    with pytest.raises(mc.McError) as e:
        mc.mc_price_qmc(ctx, model, mc.Payoff(mc.MC_BASKET_CALL, 100.0), 1000, kw.get("n", 1),
                        SEED, kw.get("R", 4),
                        mc.Options(prec=kw.get("prec", mc.MC_FP32), path_offset=kw.get("offset", 0),
                                   path_values=kw.get("pv", False)))
    assert e.value.status == status
