"""The allocation-free entry point mc_price_noalloc against mc_price: the
same kernels with the run's moments in the library's static per-GPU
scratch instead of an allocated workspace, so the results must be bit for
bit those of mc_price. Two calls in a row, the second smaller, so that the
second reads a scratch the first left behind; then the argument errors."""
import math

import pytest

import paper_1906_02818_amd as mc
import synth

pytestmark = pytest.mark.gpu
SEED = synth.SEED
KEYS = ("price", "std_err", "variance", "delta", "delta_se", "vega", "vega_se", "plain_price",
        "plain_std_err", "cv_beta", "vrf", "n_paths", "n_nonfinite")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mc.mc_create(0)
    yield c
    c.close()


def gbm():
    c = synth.ASIAN_BARRIER
    return mc.Model(kind=mc.MC_GBM, S0=c["S0"], r=c["r"], T=c["T"], sigma=c["sigma"])


def heston():
    H = synth.HESTON
    return mc.Model(kind=mc.MC_HESTON, S0=H["S0"], r=H["r"], T=H["T"], v0=H["v0"],
                    kappa=H["kappa"], theta=H["theta"], xi=H["xi"], rho=H["rho"])


def same(a, b):
    for k in KEYS:
        x, y = a[k], b[k]
        assert x == y or (isinstance(x, float) and math.isnan(x) and math.isnan(y)), (k, x, y)


CASES = [
    # GBM arithmetic Asian with the geometric-Asian control variate (its beta
    # pilot runs through the scratch too), FP32.
    ("gbm asian geo-cv fp32", gbm, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0, cv=mc.MC_CV_GEO_ASIAN),
     mc.Options(pilot_paths=1 << 18), (1 << 22, 252), (65536 + 37, 100)),
    # GBM European with pathwise delta and vega, FP64.
    ("gbm euro greeks fp64", gbm, mc.Payoff(mc.MC_EURO_CALL, 100.0),
     mc.Options(prec=mc.MC_FP64, greeks=3), (1 << 20, 64), (1001, 3)),
    # Up-and-out barrier, FP32.
    ("gbm barrier fp32", gbm, mc.Payoff(mc.MC_UO_BARRIER_CALL, 100.0, B=130.0), mc.Options(),
     (1 << 22, 252), (4099, 252)),
    # Heston Asian with forward-mode delta and d/dv0, FP32.
    ("heston tangents fp32", heston, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0),
     mc.Options(greeks=3, greeks_method=mc.MC_GREEKS_TANGENT), (1 << 20, 256), (5000, 64)),
    # Heston Asian with adjoint delta and d/dv0 (one-launch sweep, checkpoints
    # in LDS), FP32.
    ("heston adjoint fp32", heston, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0),
     mc.Options(greeks=3), (1 << 20, 256), (3001, 250)),
    # Heston price, FP32.
    ("heston price fp32", heston, mc.Payoff(mc.MC_EURO_CALL, 100.0), mc.Options(),
     (1 << 22, 256), (777, 17)),
]


@pytest.mark.parametrize("name,model,payoff,opts,big,small", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_mc_price(ctx, name, model, payoff, opts, big, small):
    for n_paths, n_steps in (big, small):
        say(name, n_paths, n_steps)
        a = mc.mc_price_noalloc(ctx, model(), payoff, n_paths, n_steps, SEED, opts)
        b = mc.mc_price(ctx, model(), payoff, n_paths, n_steps, SEED, opts)
        say(f"  noalloc {a['price']:.10f} +- {a['std_err']:.3e}; mc_price {b['price']:.10f}")
        same(a, b)
        assert a["n_paths"] == n_paths


def test_noalloc_twice_in_a_row_without_mc_price_between(ctx):
    # Back-to-back allocation-free calls: the second (smaller) run starts from
    # the first run's scratch contents and must still equal mc_price.
    f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0)
    a1 = mc.mc_price_noalloc(ctx, heston(), f, 1 << 21, 128, SEED)
    a2 = mc.mc_price_noalloc(ctx, heston(), f, 3000, 128, SEED)
    same(a1, mc.mc_price(ctx, heston(), f, 1 << 21, 128, SEED))
    same(a2, mc.mc_price(ctx, heston(), f, 3000, 128, SEED))


def test_noalloc_scratch_size_and_errors(ctx):
    assert mc.mc_noalloc_scratch_bytes() == 4 << 20
    f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0)
    # The GBM and Heston price and tangent kernels run on persistent grids,
    # so the moments of any path count fit the scratch: 2^24 Heston paths
    # with tangents.
    o = mc.Options(greeks=3, greeks_method=mc.MC_GREEKS_TANGENT)
    same(mc.mc_price_noalloc(ctx, heston(), f, 1 << 24, 16, SEED, o),
         mc.mc_price(ctx, heston(), f, 1 << 24, 16, SEED, o))
    # The adjoint takes one path per thread: at 2^24 paths its 65536 block
    # moment vectors exceed the scratch, refused before any launch.
    with pytest.raises(mc.McError) as e:
        mc.mc_price_noalloc(ctx, heston(), f, 1 << 24, 16, SEED, mc.Options(greeks=3))
    assert e.value.status == mc.MC_ERR_WORKSPACE
    bad = [
        (heston(), f, mc.Options(greeks=3), 300),          # 19 adjoint checkpoints
        (heston(), f, mc.Options(path_values=True), 16),
        (gbm(), f, mc.Options(greeks=3, greeks_method=mc.MC_GREEKS_FD_CRN), 16),
        (heston(), mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0, cv=mc.MC_CV_LEARNED),
         mc.Options(cv_weights=synth.glorot_mlp()), 16),
    ]
    for model, payoff, o, n_steps in bad:
        with pytest.raises(mc.McError) as e:
            mc.mc_price_noalloc(ctx, model, payoff, 4096, n_steps, SEED, o)
        assert e.value.status == mc.MC_ERR_UNSUPPORTED
    d = 16
    sigma, corr, _ = synth.basket_market(d)
    bm = mc.Model(kind=mc.MC_GBM_BASKET, S0=[100.0] * d, r=0.05, T=1.0, sigma=sigma, corr=corr)
    with pytest.raises(mc.McError) as e:
        mc.mc_price_noalloc(ctx, bm, mc.Payoff(mc.MC_BASKET_CALL, 100.0), 4096, 4, SEED)
    assert e.value.status == mc.MC_ERR_UNSUPPORTED
    # The failed calls leave the scratch usable.
    same(mc.mc_price_noalloc(ctx, heston(), f, 4096, 16, SEED),
         mc.mc_price(ctx, heston(), f, 4096, 16, SEED))
