"""GPU parity of the basket kernel (correlated increments Z L'^T on the
matrix cores) against the FP64 oracle, in FP32, BF16, FP16 and split-BF16
matrix precision: per-path values, aggregate prices within 2e-5 (FP32) or
0.1 standard errors (reduced precision), the full-size launch on sampled
paths, the geometric-basket closed form, ragged shapes and padding."""
import math

import numpy as np
import pytest

import oracle
import paper_1906_02818_amd as mc
import synth
from closed_forms import geo_basket_call

pytestmark = pytest.mark.gpu
SEED = synth.SEED
PRECS = {"fp32": mc.MC_FP32, "bf16": mc.MC_BF16_GEMM, "fp16": mc.MC_FP16_GEMM,
         "bf16x2": mc.MC_BF16X2_GEMM}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mc.mc_create(0)
    yield c
    c.close()


def market(d, r=0.05):
    sigma, corr, lam = synth.basket_market(d)
    L = oracle.cholesky(corr)
    S0 = np.full(d, 100.0)
    w = np.full(d, 1.0 / d)
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=S0, r=r, T=1.0, sigma=sigma, corr=corr)
    return model, S0, sigma, corr, L, w


def run(ctx, model, K, N, n, prec, offset=0, weights=None):
    return mc.mc_price(ctx, model, mc.Payoff(mc.MC_BASKET_CALL, K, weights=weights), N, n, SEED,
                       mc.Options(prec=prec, greeks=mc.MC_GREEK_DELTA, path_offset=offset,
                                  path_values=True))


@pytest.mark.parametrize("d,N,n,offset", [(32, 4096, 8, 0), (48, 1000, 5, 77), (16, 300, 3, 0),
                                          (256, 2048, 4, (1 << 32) - 100)])
@pytest.mark.parametrize("pname", list(PRECS))
def test_basket_parity_small(ctx, d, N, n, offset, pname):
    say("basket", d, N, n, offset, pname)
    model, S0, sigma, corr, L, w = market(d)
    r = run(ctx, model, 100.0, N, n, PRECS[pname], offset)
    o = oracle.basket(S0, sigma, L, w, 0.05, 1.0, 100.0, n, N, SEED, path0=offset)
    pv = r["path_values"]
    assert r["n_nonfinite"] == 0 and r["n_paths"] == N
    if pname == "fp32":
        np.testing.assert_allclose(pv[:, 0], o[:, 0], rtol=1e-4, atol=1e-4)
        np.testing.assert_allclose(pv[:, 1], o[:, 1], rtol=1e-4, atol=1e-4)
        away = np.abs(o[:, 0]) > 1e-3
        np.testing.assert_allclose(pv[away, 2], o[away, 2], rtol=1e-4, atol=1e-6)
        e = oracle.estimate(o[:, 0])
        assert abs(r["price"] - e["price"]) <= 2e-5 * e["price"] + 1e-9
    else:
        # Rounding Z and L' to 16 bits moves each path by a few 1e-3 in log
        # price; the price itself must stay within 0.1 standard errors.
        err = np.abs(pv[:, 0] - o[:, 0])
        say("  per-path max abs err", err.max())
        assert err.max() < 0.5
        e = oracle.estimate(o[:, 0])
        say(f"  price {r['price']:.6f} oracle {e['price']:.6f} se {e['std_err']:.3e} "
            f"err/se {abs(r['price'] - e['price']) / e['std_err']:.3f}")
        assert abs(r["price"] - e["price"]) < 0.1 * e["std_err"]


def test_cached_factor_follows_the_correlation_matrix(ctx):
    # The context keeps the Cholesky factor of the last correlation matrix:
    # a changed matrix is factorised again (paths against the oracle with its
    # own factor), a matrix that is not positive definite is refused, and the
    # first matrix afterwards gives bit-identical paths.
    d, N, n = 32, 2048, 4
    say("basket factor cache", d, N, n)
    model, S0, sigma, corr, L, w = market(d)
    a = run(ctx, model, 100.0, N, n, mc.MC_FP32)
    corr2 = 0.5 * corr + 0.5 * np.eye(d)
    model2 = mc.Model(kind=mc.MC_GBM_BASKET, S0=S0, r=0.05, T=1.0, sigma=sigma, corr=corr2)
    b = run(ctx, model2, 100.0, N, n, mc.MC_FP32)
    o = oracle.basket(S0, sigma, oracle.cholesky(corr2), w, 0.05, 1.0, 100.0, n, N, SEED)
    np.testing.assert_allclose(b["path_values"][:, 0], o[:, 0], rtol=1e-4, atol=1e-4)
    assert np.abs(b["path_values"][:, 0] - a["path_values"][:, 0]).max() > 1e-2
    bad = corr.copy()
    bad[0, 1] = bad[1, 0] = 1.5
    model_bad = mc.Model(kind=mc.MC_GBM_BASKET, S0=S0, r=0.05, T=1.0, sigma=sigma, corr=bad)
    for _ in range(2):
        with pytest.raises(mc.McError) as e:
            run(ctx, model_bad, 100.0, N, n, mc.MC_FP32)
        assert e.value.status == mc.MC_ERR_NOT_PD
    c = run(ctx, model, 100.0, N, n, mc.MC_FP32)
    np.testing.assert_array_equal(c["path_values"], a["path_values"])


@pytest.mark.parametrize("pname", list(PRECS))
def test_basket_full_size_sampled_paths(ctx, pname):
    # The configured workload: d = 256, 100 steps, 2^20 paths.
    c = synth.BASKET
    d, N, n = c["d"], c["n_paths"], c["n_steps"]
    say("basket full size", pname)
    model, S0, sigma, corr, L, w = market(d, c["r"])
    r = run(ctx, model, c["K"], N, n, PRECS[pname])
    pv = r["path_values"]
    assert r["n_nonfinite"] == 0 and np.all(np.isfinite(pv))
    rng = np.random.default_rng(4)
    idx = np.unique(np.concatenate([rng.choice(N, 96, replace=False), [0, 31, 32, 255, N - 1]]))
    o = np.concatenate([oracle.basket(S0, sigma, L, w, c["r"], c["T"], c["K"], n, 1, SEED,
                                      path0=int(p)) for p in idx])
    tol = 1e-4 if pname == "fp32" else 2e-2
    np.testing.assert_allclose(pv[idx, 0], o[:, 0], rtol=tol, atol=tol)
    np.testing.assert_allclose(pv[idx, 1], o[:, 1], rtol=tol, atol=tol)
    # The geometric basket is exactly lognormal under log-Euler.
    gm = pv[:, 1].mean()
    gse = pv[:, 1].std(ddof=1) / math.sqrt(N)
    ref = geo_basket_call(S0, sigma, corr, w, c["r"], c["T"], c["K"])
    say(f"  {pname}: price {r['price']:.5f} +- {r['std_err']:.5f}  geo {gm:.5f} +- {gse:.5f} "
        f"closed form {ref:.5f}  delta0 {r['delta']:.6f}  kernel {r['kernel_ms']:.2f} ms")
    assert abs(gm - ref) < 4 * gse


def test_reduced_precision_within_tenth_of_se_of_fp32_full_size(ctx):
    # Identical normals: the reduced-precision prices differ from the FP32
    # one (itself within 2e-5 of the FP64 oracle) by well under 0.1 SE.
    c = synth.BASKET
    model, *_ = market(c["d"], c["r"])
    base = mc.mc_price(ctx, model, mc.Payoff(mc.MC_BASKET_CALL, c["K"]), c["n_paths"],
                       c["n_steps"], SEED, mc.Options(prec=mc.MC_FP32))
    for pname in ("bf16", "fp16", "bf16x2"):
        r = mc.mc_price(ctx, model, mc.Payoff(mc.MC_BASKET_CALL, c["K"]), c["n_paths"],
                        c["n_steps"], SEED, mc.Options(prec=PRECS[pname]))
        dev = abs(r["price"] - base["price"]) / base["std_err"]
        say(f"  {pname}: {r['price']:.6f} vs fp32 {base['price']:.6f}: {dev:.4f} SE, "
            f"kernel {r['kernel_ms']:.2f} ms (fp32 {base['kernel_ms']:.2f} ms)")
        assert dev < 0.1
