"""GPU parity of the multilevel estimator (telescoping sum of coupled level
corrections, Sec. V-B) against the FP64 oracle on the same paths.

Time coupling (GBM): the coarse path of level l takes the normalised sums
of the fine path's normals, which is the oracle's `coarsen` argument, so
the mean and variance of every correction P_l - P_{l-1} are compared with
the same statistics of the oracle's per-path differences (FP64: 1e-9; FP32
within the single-precision tolerance). Log-Euler European corrections are
zero path by path (both grids give the same terminal value of the same
Brownian path). Precision coupling (basket BF16 -> FP32): the correction's
fine and coarse means equal the single-level prices on the same paths, and
the correction equals the FP64 oracle minus the BF16 run on those paths up
to FP32 rounding. Plus chunked levels (> 2^20 paths) and argument errors."""
import numpy as np
import pytest

import oracle
import paper_1906_02818_amd as mc
import synth

pytestmark = pytest.mark.gpu
SEED = synth.SEED
E = synth.EURO
CH = {mc.MC_EURO_CALL: 0, mc.MC_ASIAN_ARITH_CALL: 1}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mc.mc_create(0)
    yield c
    c.close()


def gbm_model(scheme):
    return mc.Model(kind=mc.MC_GBM, S0=E["S0"], r=E["r"], T=E["T"], sigma=E["sigma"],
                    scheme=scheme)


def oracle_level(scheme, kind, n_f, n_c, c, N, tag):
    """Per-path fine and coarse payoffs of one correction level."""
    args = (E["S0"], E["r"], E["sigma"], E["T"], E["K"], 1e300)
    fine = oracle.gbm(*args, n_f, N, SEED, tag=tag, scheme=scheme)[:, CH[kind]]
    coarse = oracle.gbm(*args, n_c, N, SEED, tag=tag, scheme=scheme, coarsen=c)[:, CH[kind]]
    return fine, coarse


@pytest.mark.parametrize("scheme,kind,steps,c", [
    (mc.MC_EULER_S, mc.MC_EURO_CALL, [8, 16, 32], 2),
    (mc.MC_EULER_S, mc.MC_ASIAN_ARITH_CALL, [4, 16, 64], 4),
    (mc.MC_LOG_EULER, mc.MC_ASIAN_ARITH_CALL, [8, 16], 2),
    (mc.MC_EULER_S, mc.MC_EURO_CALL, [7, 14, 28], 2),        # odd coarse step count
])
def test_time_coupling_fp64_matches_oracle(ctx, scheme, kind, steps, c):
    say("mlmc time fp64", scheme, kind, steps)
    N = 3000
    levels = [mc.Level(n, mc.MC_FP64, N) for n in steps]
    r = mc.mc_price_mlmc(ctx, gbm_model(scheme), mc.Payoff(kind, E["K"]), levels, SEED)
    args = (E["S0"], E["r"], E["sigma"], E["T"], E["K"], 1e300)
    p0 = oracle.gbm(*args, steps[0], N, SEED, tag=0, scheme=scheme)[:, CH[kind]]
    assert r["levels"][0]["coupling"] == mc.MC_COUPLE_NONE
    np.testing.assert_allclose(r["levels"][0]["mean"], p0.mean(), rtol=1e-11)
    np.testing.assert_allclose(r["levels"][0]["variance"], p0.var(ddof=1), rtol=1e-10)
    total = p0.mean()
    var_n = p0.var(ddof=1) / N
    for l in range(1, len(steps)):
        fine, coarse = oracle_level(scheme, kind, steps[l], steps[l - 1], steps[l] // steps[l - 1],
                                    N, 16 * l)
        d = fine - coarse
        lv = r["levels"][l]
        assert lv["coupling"] == mc.MC_COUPLE_TIME and lv["n_paths"] == N
        np.testing.assert_allclose(lv["fine_mean"], fine.mean(), rtol=1e-11)
        np.testing.assert_allclose(lv["coarse_mean"], coarse.mean(), rtol=1e-11)
        np.testing.assert_allclose(lv["mean"], d.mean(), rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(lv["variance"], d.var(ddof=1), rtol=1e-9, atol=1e-20)
        total += d.mean()
        var_n += d.var(ddof=1) / N
    np.testing.assert_allclose(r["price"], total, rtol=1e-10)
    np.testing.assert_allclose(r["std_err"], np.sqrt(var_n), rtol=1e-8)


def test_time_coupling_fp32_matches_oracle(ctx):
    say("mlmc time fp32")
    N, steps = 4096, [16, 64]
    kind = mc.MC_ASIAN_ARITH_CALL
    levels = [mc.Level(n, mc.MC_FP32, N) for n in steps]
    r = mc.mc_price_mlmc(ctx, gbm_model(mc.MC_LOG_EULER), mc.Payoff(kind, E["K"]), levels, SEED)
    fine, coarse = oracle_level(mc.MC_LOG_EULER, kind, 64, 16, 4, N, 16)
    lv = r["levels"][1]
    scale = fine.mean()
    assert abs(lv["fine_mean"] - fine.mean()) <= 2e-5 * scale
    assert abs(lv["coarse_mean"] - coarse.mean()) <= 2e-5 * scale
    assert abs(lv["mean"] - (fine - coarse).mean()) <= 2e-5 * scale
    np.testing.assert_allclose(lv["variance"], (fine - coarse).var(ddof=1), rtol=2e-3)


def test_log_euler_european_correction_vanishes(ctx):
    # Same Brownian path on both grids: ln S_T is identical, so every path's
    # European payoff difference is rounding only.
    say("mlmc log euro zero")
    levels = [mc.Level(8, mc.MC_FP64, 4096), mc.Level(16, mc.MC_FP64, 4096),
              mc.Level(64, mc.MC_FP64, 4096)]
    r = mc.mc_price_mlmc(ctx, gbm_model(mc.MC_LOG_EULER), mc.Payoff(mc.MC_EURO_CALL, E["K"]),
                         levels, SEED)
    for lv in r["levels"][1:]:
        assert abs(lv["mean"]) < 1e-12 and lv["variance"] < 1e-24


def test_euler_s_correction_variance_decays(ctx):
    # Strong order 1/2 of Euler on S: Var(P_l - P_{l-1}) ~ dt, halving with
    # each doubling of the steps (the multilevel variance decay).
    say("mlmc variance decay")
    steps = [8, 16, 32, 64, 128]
    levels = [mc.Level(n, mc.MC_FP32, 1 << 18) for n in steps]
    r = mc.mc_price_mlmc(ctx, gbm_model(mc.MC_EULER_S), mc.Payoff(mc.MC_EURO_CALL, E["K"]),
                         levels, SEED)
    v = [lv["variance"] for lv in r["levels"][1:]]
    for a, b in zip(v, v[1:]):
        assert 1.6 < a / b < 2.5, v


def test_precision_coupling_basket(ctx):
    say("mlmc basket precision")
    d, n, N = 32, 10, 8192
    sigma, corr, _ = synth.basket_market(d)
    L = oracle.cholesky(corr)
    S0 = np.full(d, 100.0)
    w = np.full(d, 1.0 / d)
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=S0, r=0.05, T=1.0, sigma=sigma, corr=corr)
    f = mc.Payoff(mc.MC_BASKET_CALL, 100.0)
    levels = [mc.Level(n, mc.MC_BF16_GEMM, N), mc.Level(n, mc.MC_FP32, N)]
    r = mc.mc_price_mlmc(ctx, model, f, levels, SEED)
    lv = r["levels"][1]
    assert lv["coupling"] == mc.MC_COUPLE_PRECISION
    lo = mc.mc_price(ctx, model, f, N, n, SEED, mc.Options(prec=mc.MC_BF16_GEMM, stream_tag=16))
    hi = mc.mc_price(ctx, model, f, N, n, SEED, mc.Options(prec=mc.MC_FP32, stream_tag=16))
    base = mc.mc_price(ctx, model, f, N, n, SEED, mc.Options(prec=mc.MC_BF16_GEMM))
    np.testing.assert_allclose(lv["fine_mean"], hi["price"], rtol=1e-12)
    np.testing.assert_allclose(lv["coarse_mean"], lo["price"], rtol=1e-12)
    np.testing.assert_allclose(lv["mean"], hi["price"] - lo["price"], rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(r["levels"][0]["mean"], base["price"], rtol=1e-14)
    # The correction is the reference-precision price minus the BF16 one on
    # the same paths: the FP64 oracle stands in for FP32 to within 1e-4.
    o = oracle.basket(S0, sigma, L, w, 0.05, 1.0, 100.0, n, N, SEED, tag=16)[:, 0]
    assert abs(lv["mean"] - (o.mean() - lv["coarse_mean"])) < 1e-4 * o.mean()
    assert lv["variance"] < 1e-3 * r["levels"][0]["variance"]


def test_chunked_level_matches_single_runs(ctx):
    # A correction level above 2^20 paths runs in chunks; its fine and
    # coarse means must equal single runs over the whole path range.
    say("mlmc chunked")
    N = (1 << 20) + 3
    model = gbm_model(mc.MC_LOG_EULER)
    f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, E["K"])
    levels = [mc.Level(4, mc.MC_FP32, 1024), mc.Level(8, mc.MC_FP32, N)]
    r = mc.mc_price_mlmc(ctx, model, f, levels, SEED, mc.Options(path_offset=5))
    fine = mc.mc_price(ctx, model, f, N, 8, SEED, mc.Options(stream_tag=16, path_offset=5))
    lv = r["levels"][1]
    assert lv["n_paths"] == N
    np.testing.assert_allclose(lv["fine_mean"], fine["price"], rtol=1e-12)


@pytest.mark.parametrize("levels,model_kind,payoff,status", [
    ([mc.Level(8, mc.MC_FP32, 64), mc.Level(16, mc.MC_FP64, 64)], mc.MC_GBM,
     mc.Payoff(mc.MC_EURO_CALL, 100.0), mc._abi.MC_ERR_UNSUPPORTED),
    ([mc.Level(8, mc.MC_FP32, 64), mc.Level(24, mc.MC_FP32, 64)], mc.MC_GBM,
     mc.Payoff(mc.MC_EURO_CALL, 100.0), mc._abi.MC_ERR_UNSUPPORTED),
    ([mc.Level(8, mc.MC_FP32, 64), mc.Level(16, mc.MC_FP32, 64)], mc.MC_HESTON,
     mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0), mc._abi.MC_ERR_UNSUPPORTED),
    ([mc.Level(8, mc.MC_FP32, 64), mc.Level(16, mc.MC_FP32, 64)], mc.MC_GBM,
     mc.Payoff(mc.MC_UO_BRIDGE_CALL, 100.0, B=130.0), mc._abi.MC_ERR_UNSUPPORTED),
    ([mc.Level(8, mc.MC_FP32, 1)], mc.MC_GBM, mc.Payoff(mc.MC_EURO_CALL, 100.0),
     mc._abi.MC_ERR_INVALID_ARG),
    ([mc.Level(8, mc.MC_FP32, 64)] * 9, mc.MC_GBM, mc.Payoff(mc.MC_EURO_CALL, 100.0),
     mc._abi.MC_ERR_INVALID_ARG),
    ([mc.Level(8, mc.MC_FP32, 64)], mc.MC_GBM,
     mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0, cv=mc.MC_CV_GEO_ASIAN), mc._abi.MC_ERR_UNSUPPORTED),
])
def test_mlmc_argument_errors(ctx, levels, model_kind, payoff, status):
    if model_kind == mc.MC_GBM:
        model = gbm_model(mc.MC_LOG_EULER)
    else:
        H = synth.HESTON
        model = mc.Model(kind=mc.MC_HESTON, S0=H["S0"], r=H["r"], T=H["T"], v0=H["v0"],
                         kappa=H["kappa"], theta=H["theta"], xi=H["xi"], rho=H["rho"])
    with pytest.raises(mc.McError) as e:
        mc.mc_price_mlmc(ctx, model, payoff, levels, SEED)
    assert e.value.status == status


def test_heston_precision_coupling(ctx):
    # FP32 -> FP64 correction on Heston: the FP64 level matches the oracle
    # path for path, so the correction is the FP32 rounding effect only.
    say("mlmc heston precision")
    H = synth.HESTON
    model = mc.Model(kind=mc.MC_HESTON, S0=H["S0"], r=H["r"], T=H["T"], v0=H["v0"],
                     kappa=H["kappa"], theta=H["theta"], xi=H["xi"], rho=H["rho"])
    N, n = 2048, 32
    f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, H["K"])
    r = mc.mc_price_mlmc(ctx, model, f, [mc.Level(n, mc.MC_FP32, N), mc.Level(n, mc.MC_FP64, N)],
                         SEED)
    o = oracle.heston(H["S0"], H["v0"], H["kappa"], H["theta"], H["xi"], H["rho"], H["r"],
                      H["T"], H["K"], n, N, SEED, tag=16)[:, 1]
    lv = r["levels"][1]
    np.testing.assert_allclose(lv["fine_mean"], o.mean(), rtol=1e-11)
    assert abs(lv["mean"]) < 2e-5 * o.mean()
