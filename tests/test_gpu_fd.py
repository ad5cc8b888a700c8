"""Finite-difference greeks on common random numbers (MC_GREEKS_FD_CRN): the
only route to greeks of discontinuous payoffs (barriers), where pathwise
derivatives do not exist.

* European GBM: delta and vega against the Black-Scholes closed forms, and
  against the pathwise tangents on the same paths; more than 2^20 paths,
  so the per-path values pass through several device chunks, whose result
  must equal the mean of the per-path differences of two explicit bumped
  runs exactly.
* Discrete and Brownian-bridge up-and-out calls: against the oracle's own
  central differences on the same paths (FP64, same seed and tags); the
  bumped pairs run with FP64 paths, so the knock-out decisions agree.
* Heston: delta and d/dv0 against the oracle's differences.
* Basket: delta of asset 0 against the pathwise delta.
* The method is reported in the result; argument errors.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1906_02818_amd as mc
import synth
from closed_forms import bs_delta, bs_vega

pytestmark = pytest.mark.gpu
SEED = synth.SEED
H_REL = 1e-3
FD = mc.MC_GREEK_DELTA | mc.MC_GREEK_VEGA


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mc.mc_create(0)
    yield c
    c.close()


def gbm(S0=100.0, sigma=0.25, r=0.03):
    return mc.Model(kind=mc.MC_GBM, S0=S0, r=r, T=1.0, sigma=sigma)


def fd_opts(**kw):
    return mc.Options(greeks=FD, greeks_method=mc.MC_GREEKS_FD_CRN, fd_rel_step=H_REL, **kw)


def test_european_fd_matches_closed_form_and_pathwise(ctx):
    N, n = (1 << 20) + 5, 64
    f = mc.Payoff(mc.MC_EURO_CALL, 100.0)
    r = mc.mc_price(ctx, gbm(), f, N, n, SEED, fd_opts())
    pw = mc.mc_price(ctx, gbm(), f, N, n, SEED, mc.Options(greeks=FD))
    assert r["greeks_method"] == mc.MC_GREEKS_FD_CRN
    assert pw["greeks_method"] == mc.MC_GREEKS_PATHWISE
    assert r["price"] == pw["price"]
    d, v = bs_delta(100.0, 100.0, 0.03, 0.25, 1.0), bs_vega(100.0, 100.0, 0.03, 0.25, 1.0)
    say(f"  delta fd {r['delta']:.6f} +- {r['delta_se']:.1e} pathwise {pw['delta']:.6f} bs {d:.6f}")
    say(f"  vega  fd {r['vega']:.5f} +- {r['vega_se']:.1e} pathwise {pw['vega']:.5f} bs {v:.5f}")
    assert abs(r["delta"] - d) < 4 * r["delta_se"] + 1e-4
    assert abs(r["vega"] - v) < 4 * r["vega_se"] + 1e-3
    # FP32 pathwise tangents against FP64 differences on the same paths: they
    # differ on the paths whose terminal price lies within the bump of the
    # strike, and by the pathwise tangents' FP32 rounding.
    assert abs(r["delta"] - pw["delta"]) < 0.2 * pw["delta_se"]
    assert abs(r["vega"] - pw["vega"]) < 0.2 * pw["vega_se"]


def test_fd_equals_explicit_bumped_runs_across_chunks(ctx):
    N, n = (1 << 20) + 777, 16
    f = mc.Payoff(mc.MC_UO_BARRIER_CALL, 100.0, B=130.0)
    r = mc.mc_price(ctx, gbm(), f, N, n, SEED, fd_opts(path_offset=123))
    col = mc.mc_path_channels(gbm(), f, mc.Options(prec=mc.MC_FP64)).index("uo")
    # The bumped pairs run with FP64 paths.
    o64 = mc.Options(prec=mc.MC_FP64, path_values=True, path_offset=123)
    up = mc.mc_price(ctx, gbm(S0=100.0 * (1 + H_REL)), f, N, n, SEED, o64)["path_values"][:, col]
    dn = mc.mc_price(ctx, gbm(S0=100.0 * (1 - H_REL)), f, N, n, SEED, o64)["path_values"][:, col]
    diff = (up - dn) / (2 * H_REL * 100.0)
    assert r["delta"] == pytest.approx(diff.mean(), rel=1e-12, abs=1e-15)
    assert r["delta_se"] == pytest.approx(diff.std(ddof=1) / math.sqrt(N), rel=1e-9)


@pytest.mark.parametrize("kind,ch", [(mc.MC_UO_BARRIER_CALL, 3), (mc.MC_UO_BRIDGE_CALL, 9)])
def test_barrier_fd_matches_oracle_differences(ctx, kind, ch):
    N, n, S0, sig, r_, K, B = 1 << 16, 64, 100.0, 0.25, 0.03, 100.0, 130.0
    f = mc.Payoff(kind, K, B=B)
    r = mc.mc_price(ctx, gbm(), f, N, n, SEED, fd_opts())
    assert r["greeks_method"] == mc.MC_GREEKS_FD_CRN

    def orc(S, s):
        return oracle.gbm(S, r_, s, 1.0, K, B, n, N, SEED)[:, ch]
    od = (orc(S0 * (1 + H_REL), sig) - orc(S0 * (1 - H_REL), sig)) / (2 * H_REL * S0)
    ov = (orc(S0, sig * (1 + H_REL)) - orc(S0, sig * (1 - H_REL))) / (2 * H_REL * sig)
    for key, o in (("delta", od), ("vega", ov)):
        se = o.std(ddof=1) / math.sqrt(N)
        say(f"  {key}: gpu {r[key]:.6f} +- {r[key + '_se']:.2e} oracle {o.mean():.6f} +- {se:.2e}")
        # FP64 bumped paths on both sides: the same knock-out decisions.
        assert r[key] == pytest.approx(o.mean(), rel=1e-7, abs=1e-9)
        assert r[key + "_se"] == pytest.approx(se, rel=1e-6)


def test_heston_fd_matches_oracle_differences(ctx):
    Hs = synth.HESTON
    N, n = 1 << 15, 64
    p = {k: Hs[k] for k in ("S0", "v0", "kappa", "theta", "xi", "rho", "r", "T", "K")}

    def model(**over):
        q = dict(p, **over)
        return mc.Model(kind=mc.MC_HESTON, S0=q["S0"], r=q["r"], T=q["T"], v0=q["v0"],
                        kappa=q["kappa"], theta=q["theta"], xi=q["xi"], rho=q["rho"])
    f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, p["K"])
    r = mc.mc_price(ctx, model(), f, N, n, SEED, fd_opts())

    def orc(**over):
        q = dict(p, **over)
        return oracle.heston(q["S0"], q["v0"], q["kappa"], q["theta"], q["xi"], q["rho"], q["r"],
                             q["T"], q["K"], n, N, SEED)[:, 1]
    od = (orc(S0=p["S0"] * (1 + H_REL)) - orc(S0=p["S0"] * (1 - H_REL))) / (2 * H_REL * p["S0"])
    ov = (orc(v0=p["v0"] * (1 + H_REL)) - orc(v0=p["v0"] * (1 - H_REL))) / (2 * H_REL * p["v0"])
    for key, o in (("delta", od), ("vega", ov)):
        se = o.std(ddof=1) / math.sqrt(N)
        say(f"  {key}: gpu {r[key]:.6f} +- {r[key + '_se']:.2e} oracle {o.mean():.6f} +- {se:.2e}")
        assert r[key] == pytest.approx(o.mean(), rel=1e-6, abs=1e-9)
        assert r[key + "_se"] == pytest.approx(se, rel=1e-5)


def test_basket_fd_delta_matches_pathwise(ctx):
    d = 16
    sigma, corr, _ = synth.basket_market(d)
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=np.full(d, 100.0), r=0.05, T=1.0, sigma=sigma,
                     corr=corr)
    f = mc.Payoff(mc.MC_BASKET_CALL, 100.0)
    N, n = 1 << 17, 8
    r = mc.mc_price(ctx, model, f, N, n, SEED,
                    mc.Options(greeks=mc.MC_GREEK_DELTA, greeks_method=mc.MC_GREEKS_FD_CRN))
    pw = mc.mc_price(ctx, model, f, N, n, SEED, mc.Options(greeks=mc.MC_GREEK_DELTA))
    say(f"  basket delta0 fd {r['delta']:.6f} +- {r['delta_se']:.1e} pathwise {pw['delta']:.6f}")
    assert abs(r["delta"] - pw["delta"]) < 0.2 * pw["delta_se"]


def test_fd_argument_errors(ctx):
    f = mc.Payoff(mc.MC_UO_BARRIER_CALL, 100.0, B=130.0)

    def status(model=None, **kw):
        with pytest.raises(mc.McError) as e:
            mc.mc_price(ctx, model or gbm(), f, 1024, 8, SEED, mc.Options(**kw))
        return str(e.value)
    # Pathwise greeks of a barrier do not exist.
    assert "UNSUPPORTED" in status(greeks=FD)
    for h in (0.0, 0.5, -1e-3, float("nan")):
        assert "INVALID_ARG" in status(greeks=FD, greeks_method=mc.MC_GREEKS_FD_CRN,
                                       fd_rel_step=h)
    assert "INVALID_ARG" in status(greeks=FD, greeks_method=7)
    assert "INVALID_ARG" in status(model=gbm(sigma=0.0), greeks=mc.MC_GREEK_VEGA,
                                   greeks_method=mc.MC_GREEKS_FD_CRN)
    d = 16
    sigma, corr, _ = synth.basket_market(d)
    basket = mc.Model(kind=mc.MC_GBM_BASKET, S0=np.full(d, 100.0), r=0.05, T=1.0, sigma=sigma,
                      corr=corr)
    with pytest.raises(mc.McError) as e:
        mc.mc_price(ctx, basket, mc.Payoff(mc.MC_BASKET_CALL, 100.0), 1024, 4, SEED,
                    mc.Options(greeks=mc.MC_GREEK_VEGA, greeks_method=mc.MC_GREEKS_FD_CRN))
    assert "UNSUPPORTED" in str(e.value)
