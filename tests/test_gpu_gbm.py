"""GPU parity of the GBM path kernel against the FP64 oracle: Philox words
and normals, per-path payoff channels, aggregate prices, the full-size launch
on sampled paths, ragged shapes, sharding and determinism. Every call goes
through the C ABI (libmcpath.so)."""
import math

import numpy as np
import pytest

import oracle
import paper_1906_02818_amd as mc
import synth
from closed_forms import arith_asian2_call, bs_call, bs_delta, bs_vega, geo_asian_call

pytestmark = pytest.mark.gpu

SEED = synth.SEED


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mc.mc_create(0)
    yield c
    c.close()


def gbm_model(c, scheme=mc.MC_LOG_EULER):
    return mc.Model(kind=mc.MC_GBM, S0=c["S0"], r=c["r"], T=c["T"], sigma=c["sigma"],
                    scheme=scheme)


# ---------------------------------------------------------------- RNG ----
def test_philox_words_bit_exact(ctx):
    rng = np.random.default_rng(1)
    n = 20000
    paths = rng.integers(0, 2**63, n, dtype=np.uint64) * np.uint64(2)
    paths[:100] = np.arange(100, dtype=np.uint64)
    blocks = rng.integers(0, 2**32, n, dtype=np.uint64)
    for seed in (SEED, (0xDEADBEEF << 32) | 7):
        for tag in (0, 1, 5, 0xFFFFFFFF):
            say("philox words", seed, tag)
            got = mc.mc_philox_words(ctx, seed, tag, paths, blocks)
            want = oracle.words(seed, tag, paths, blocks)
            assert np.array_equal(got, want)


def test_normals_match_oracle(ctx):
    for path, k0 in ((0, 0), (123456789, 1001), ((1 << 40) + 5, 3)):
        say("normals", path, k0)
        ref = oracle.normals(SEED, 0, path, k0, 8192)
        z64 = mc.mc_normals(ctx, SEED, 0, path, k0, 8192, mc.MC_FP64)
        np.testing.assert_allclose(z64, ref, rtol=1e-13, atol=1e-13)
        z32 = mc.mc_normals(ctx, SEED, 0, path, k0, 8192, mc.MC_FP32)
        err = np.abs(z32 - ref) / (1.0 + np.abs(ref))
        say("  fp32 normal max err", err.max())
        assert err.max() < 4e-6


# ------------------------------------------------------ European (FP64) --
def test_european_fp64_full_size_parity_and_closed_form(ctx):
    c = synth.EURO
    N, n = c["n_paths"], c["n_steps"]
    say("euro fp64", N, n)
    r = mc.mc_price(ctx, gbm_model(c), mc.Payoff(mc.MC_EURO_CALL, c["K"]), N, n, SEED,
                    mc.Options(prec=mc.MC_FP64, greeks=3, path_values=True))
    assert r["path_channels"] == ["euro", "euro_delta", "euro_vega"]
    o = oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], 1e300, n, N, SEED)
    ref = o[:, [0, 4, 5]]
    pv = r["path_values"]
    np.testing.assert_allclose(pv, ref, rtol=1e-12, atol=1e-11)
    for col, key in ((0, "price"), (1, "delta"), (2, "vega")):
        e = oracle.estimate(ref[:, col])
        assert abs(r[key] - e["price"]) <= 1e-12 * abs(e["price"]), key
    e = oracle.estimate(ref[:, 0])
    assert abs(r["std_err"] - e["std_err"]) <= 1e-10 * e["std_err"]
    args = (c["S0"], c["K"], c["r"], c["sigma"], c["T"])
    assert abs(r["price"] - bs_call(*args)) < 4 * r["std_err"]
    assert abs(r["delta"] - bs_delta(*args)) < 4 * r["delta_se"]
    assert abs(r["vega"] - bs_vega(*args)) < 4 * r["vega_se"]
    say("  price", r["price"], "+-", r["std_err"], "BS", bs_call(*args), "kernel ms", r["kernel_ms"])


def test_european_fp32_within_2e5_of_oracle(ctx):
    c = synth.EURO
    N, n = c["n_paths"], c["n_steps"]
    say("euro fp32", N, n)
    r = mc.mc_price(ctx, gbm_model(c), mc.Payoff(mc.MC_EURO_CALL, c["K"]), N, n, SEED,
                    mc.Options(prec=mc.MC_FP32, greeks=3, path_values=True))
    o = oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], 1e300, n, N, SEED)
    for col, key in ((0, "price"), (4, "delta"), (5, "vega")):
        e = oracle.estimate(o[:, col])
        rel = abs(r[key] - e["price"]) / abs(e["price"])
        say(f"  {key} rel err vs oracle {rel:.2e}")
        assert rel < 2e-5
    pv = r["path_values"]
    away = np.abs(o[:, 0]) > 1e-3          # not at the kink S_T = K
    err = np.abs(pv[away, 0] - o[away, 0]) / (1 + np.abs(o[away, 0]))
    assert err.max() < 2e-4


# ------------------------------------------- Asian + barrier + geometric --
def _asian_barrier_check(r, o, tol_rel=2e-5):
    pv = r["path_values"]                 # asian, geo, uo
    res = {}
    for j, oc in ((0, 1), (1, 2)):
        away = np.abs(o[:, oc]) > 1e-3
        err = np.abs(pv[away, j] - o[away, oc]) / (1.0 + np.abs(o[away, oc]))
        res[oc] = err.max()
        assert err.max() < 3e-4, (oc, err.max())
    # Knock-out decisions agree except where the oracle's margin is within
    # FP32 resolution of the barrier; there either decision is valid.
    itm = o[:, 0] > 0
    ambiguous = np.abs(o[:, 10]) < 2e-5
    gpu_alive = pv[:, 2] > 0
    orc_alive = o[:, 3] > 0
    mismatch = itm & (gpu_alive != orc_alive)
    assert not np.any(mismatch & ~ambiguous)
    ok_val = np.isclose(pv[:, 2], 0.0) | (np.abs(pv[:, 2] - o[:, 0]) <= 3e-4 * (1 + o[:, 0]))
    assert np.all(ok_val[itm])
    return res, int(mismatch.sum())


def test_asian_barrier_fp32_parity_small(ctx):
    c = synth.ASIAN_BARRIER
    N, n = 1 << 16, c["n_steps"]
    say("asian/barrier fp32", N, n)
    model = gbm_model(c)
    pays = [mc.Payoff(mc.MC_ASIAN_ARITH_CALL, c["K"], cv=mc.MC_CV_GEO_ASIAN)]
    r = mc.mc_price(ctx, model, pays[0], N, n, SEED,
                    mc.Options(cv_beta=1.0, path_values=True))
    assert r["path_channels"] == ["asian", "geo", "uo"]
    o = oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], c["B"], n, N, SEED)
    # The uo channel of this instantiation uses B = +inf here (no barrier given).
    pv = r["path_values"]
    for j, oc in ((0, 1), (1, 2)):
        e = oracle.estimate(o[:, oc])
        rel = abs(pv[:, j].mean() - e["price"]) / e["price"]
        say(f"  channel {oc} rel err {rel:.2e}")
        assert rel < 2e-5
    # Plain and CV prices from the moments.
    e = oracle.estimate(o[:, 1])
    assert abs(r["plain_price"] - e["price"]) < 2e-5 * e["price"]
    cv = oracle.cv_estimate(o[:, 1], o[:, 2], geo_asian_call(c["S0"], c["K"], c["r"], c["sigma"],
                                                             c["T"], n), 1.0)
    assert abs(r["price"] - cv["price"]) < 2e-5 * cv["price"]
    assert abs(r["std_err"] - cv["std_err"]) < 1e-3 * cv["std_err"]
    # Barrier on the same paths through mc_price_multi.
    payoffs = [mc.Payoff(mc.MC_ASIAN_ARITH_CALL, c["K"]),
               mc.Payoff(mc.MC_UO_BARRIER_CALL, c["K"], B=c["B"]),
               mc.Payoff(mc.MC_ASIAN_GEO_CALL, c["K"])]
    rs = mc.mc_price_multi(ctx, model, payoffs, N, n, SEED)
    r2 = mc.mc_price(ctx, model, payoffs[1], N, n, SEED, mc.Options(path_values=True))
    assert r2["path_channels"] == ["asian", "geo", "uo"]
    res, nflip = _asian_barrier_check(r2, o)
    say("  per-path max rel err", res, "barrier flips", nflip)
    eb = oracle.estimate(np.where(np.abs(o[:, 10]) < 2e-5, r2["path_values"][:, 2], o[:, 3]))
    assert abs(rs[1]["price"] - eb["price"]) < 2e-5 * eb["price"]
    assert abs(rs[0]["price"] - oracle.estimate(o[:, 1])["price"]) < 2e-5 * e["price"]
    assert abs(rs[2]["price"] - oracle.estimate(o[:, 2])["price"]) < 2e-5 * e["price"]


def test_asian_barrier_full_size_sampled_paths(ctx):
    # The launch the benchmark times: 2^24 paths x 252 steps, one pass for the
    # Asian, the geometric Asian and the up-and-out call.
    c = synth.ASIAN_BARRIER
    N, n = c["n_paths"], c["n_steps"]
    say("asian/barrier full size", N, n)
    model = gbm_model(c)
    r = mc.mc_price(ctx, model, mc.Payoff(mc.MC_UO_BARRIER_CALL, c["K"], B=c["B"]), N, n, SEED,
                    mc.Options(path_values=True))
    pv = r["path_values"]
    assert pv.shape == (N, 3) and np.all(np.isfinite(pv))
    rng = np.random.default_rng(9)
    idx = np.unique(np.concatenate([rng.choice(N, 3000, replace=False),
                                    [0, 1, 255, 256, N - 257, N - 1]]))
    o = np.concatenate([oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], c["B"], n, 1,
                                   SEED, path0=int(p)) for p in idx])
    sub = {"path_values": pv[idx]}
    res, nflip = _asian_barrier_check(sub, o)
    say("  sampled max rel err", res, "flips", nflip)
    # Properties at full size: geometric Asian matches its closed form (log-
    # Euler is exact in law); arithmetic >= geometric; knock-out <= European.
    geo = pv[:, 1].mean()
    se = pv[:, 1].std(ddof=1) / math.sqrt(N)
    cg = geo_asian_call(c["S0"], c["K"], c["r"], c["sigma"], c["T"], n)
    say("  geo", geo, "+-", se, "closed form", cg)
    assert abs(geo - cg) < 4 * se
    assert np.all(pv[:, 0] >= pv[:, 1] - 1e-3)
    # The estimate and its standard error from the block moments (8192
    # blocks: merged in two stages, chunks of 2048 blocks, then the chunk
    # heads) against the per-path values.
    assert abs(r["price"] - pv[:, 2].mean()) < 1e-9 * r["price"]
    se_path = pv[:, 2].std(ddof=1) / math.sqrt(N)
    say("  se merged", r["std_err"], "per-path", se_path)
    assert abs(r["std_err"] / se_path - 1.0) < 1e-9


def test_geometric_control_variate_with_pilot(ctx):
    c = synth.ASIAN_BARRIER
    model = gbm_model(c)
    f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, c["K"], cv=mc.MC_CV_GEO_ASIAN)
    r = mc.mc_price(ctx, model, f, 1 << 22, c["n_steps"], SEED, mc.Options(pilot_paths=1 << 18))
    say("  cv", r["price"], r["std_err"], "plain", r["plain_price"], r["plain_std_err"],
        "beta", r["cv_beta"], "vrf", r["vrf"])
    assert 1.0 < r["cv_beta"] < 1.1
    assert r["vrf"] > 300
    assert abs(r["price"] - r["plain_price"]) < 3 * r["plain_std_err"]



def test_geometric_control_variate_in_sample(ctx):
    # MC_PILOT_IN_SAMPLE: beta = Cov(A, G) / Var(G) from the priced paths
    # themselves and the price A - beta (G - C_G) on the same paths, both
    # against the oracle's per-path values (FP64 paths, ragged path count).
    c = synth.ASIAN_BARRIER
    N, n = (1 << 16) + 37, 64
    model = gbm_model(c)
    f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, c["K"], cv=mc.MC_CV_GEO_ASIAN)
    r = mc.mc_price(ctx, model, f, N, n, SEED,
                    mc.Options(prec=mc.MC_FP64, pilot_paths=mc.MC_PILOT_IN_SAMPLE))
    o = oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], 1e300, n, N, SEED)
    beta = oracle.cv_beta(o[:, 1], o[:, 2])
    est = oracle.cv_estimate(o[:, 1], o[:, 2],
                             geo_asian_call(c["S0"], c["K"], c["r"], c["sigma"], c["T"], n), beta)
    say("  beta gpu", r["cv_beta"], "oracle", beta, "price", r["price"], est["price"])
    assert abs(r["cv_beta"] / beta - 1.0) < 1e-9
    assert abs(r["price"] - est["price"]) < 1e-10 * est["price"]
    assert abs(r["std_err"] / est["std_err"] - 1.0) < 1e-6


@pytest.mark.parametrize("K", [90.0, 115.0])
def test_arithmetic_asian_two_fixings_against_semi_closed_form(ctx, K):
    # The GPU's arithmetic Asian at K > 0 with volatility, two fixings, FP32
    # paths: within 4 standard errors of the semi-closed form (inner
    # Black-Scholes given S(T/2), quadrature over the first half).
    c = synth.ASIAN_BARRIER
    model = gbm_model(c)
    r = mc.mc_price(ctx, model, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, K), 1 << 22, 2, SEED)
    ref = arith_asian2_call(c["S0"], K, c["r"], c["sigma"], c["T"])
    say("  asian n=2", r["price"], "+-", r["std_err"], "semi-closed form", ref)
    assert abs(r["price"] - ref) < 4 * r["std_err"]

# ----------------------------------------------------------- edge cases --
@pytest.mark.parametrize("N,n,offset,scheme,prec", [
    (1000, 7, 0, mc.MC_LOG_EULER, mc.MC_FP32),
    (2, 1, 0, mc.MC_LOG_EULER, mc.MC_FP32),
    (257, 5, (1 << 32) - 3, mc.MC_LOG_EULER, mc.MC_FP64),
    (3000, 13, 12345, mc.MC_EULER_S, mc.MC_FP64),
    (3000, 13, 0, mc.MC_EULER_S, mc.MC_FP32),
    (4096, 64, 0, mc.MC_LOG_EULER, mc.MC_FP64),
])
def test_all_channels_ragged_shapes(ctx, N, n, offset, scheme, prec):
    say("ragged", N, n, offset, scheme, prec)
    S0, r_, sig, T, K, B = 100.0, 0.03, 0.25, 1.0, 100.0, 130.0
    model = mc.Model(kind=mc.MC_GBM, S0=S0, r=r_, T=T, sigma=sig, scheme=scheme)
    want_bridge = scheme == mc.MC_LOG_EULER
    kind = mc.MC_UO_BRIDGE_CALL if want_bridge else mc.MC_UO_BARRIER_CALL
    # Bridge (or plain barrier for Euler-S) selects the all-channel kernel.
    opts = mc.Options(prec=prec, path_offset=offset, path_values=True)
    res = mc.mc_price(ctx, model, mc.Payoff(kind, K, B=B), N, n, SEED, opts)
    names = res["path_channels"]
    pv = res["path_values"]
    o = oracle.gbm(S0, r_, sig, T, K, B, n, N, SEED, path0=offset,
                   scheme=0 if scheme == mc.MC_LOG_EULER else 1)
    col = {"euro": 0, "asian": 1, "geo": 2, "uo": 3, "euro_delta": 4, "euro_vega": 5,
           "asian_delta": 6, "asian_vega": 7, "uo_bridge": 9}
    rtol = 1e-11 if prec == mc.MC_FP64 else 3e-4
    for j, name in enumerate(names):
        ref = o[:, col[name]]
        if name in ("uo", "uo_bridge"):
            marg = o[:, 10 if name == "uo" else 11]
            ok = (np.abs(marg) < (1e-9 if prec == mc.MC_FP64 else 2e-5)) | \
                 (np.abs(pv[:, j] - ref) <= rtol * (1 + np.abs(ref)))
            assert np.all(ok), name
            continue
        kink = {"euro_delta": 0, "euro_vega": 0, "asian_delta": 1, "asian_vega": 1}
        if name in kink:
            away = np.abs(o[:, kink[name]]) > (1e-9 if prec == mc.MC_FP64 else 1e-3)
        else:
            away = np.ones(N, bool)
        np.testing.assert_allclose(pv[away, j], ref[away], rtol=rtol, atol=rtol, err_msg=name)


def test_sharding_merges_exactly_and_runs_are_deterministic(ctx):
    c = synth.ASIAN_BARRIER
    model = gbm_model(c)
    f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, c["K"])
    N, n = 1 << 20, 64
    a = mc.mc_price(ctx, model, f, N, n, SEED)
    b = mc.mc_price(ctx, model, f, N, n, SEED)
    assert a["price"] == b["price"] and a["std_err"] == b["std_err"]
    lo = mc.mc_price(ctx, model, f, N // 2 + 77, n, SEED)
    hi = mc.mc_price(ctx, model, f, N - (N // 2 + 77), n, SEED,
                     mc.Options(path_offset=N // 2 + 77))
    merged = (lo["price"] * lo["n_paths"] + hi["price"] * hi["n_paths"]) / N
    assert abs(merged - a["price"]) < 1e-12 * a["price"]
    # Stream tags are independent streams.
    t1 = mc.mc_price(ctx, model, f, N, n, SEED, mc.Options(stream_tag=1))
    assert t1["price"] != a["price"]
    assert abs(t1["price"] - a["price"]) < 5 * math.hypot(a["std_err"], t1["std_err"])


def test_near_perfect_control_variate_variance(ctx):
    # The estimator's variance from the merged (count, mean, co-moment)
    # vectors keeps its digits when the control variate leaves almost no
    # variance: arithmetic Asian with the geometric-Asian control variate,
    # deep in the money (both payoffs linear in the averages), r = 0 (so the
    # two averages agree to first order in sigma) and sigma = 0.005: they
    # differ by O(sigma^2). FP64 paths, a fixed coefficient. Against the
    # oracle's per-path values on the same paths with a two-pass variance:
    # VRF above 10^6, variance within 1e-6.
    S0, r_, sig, T, K, n, N = 100.0, 0.0, 0.005, 1.0, 90.0, 64, 1 << 18
    model = mc.Model(kind=mc.MC_GBM, S0=S0, r=r_, T=T, sigma=sig)
    o = oracle.gbm(S0, r_, sig, T, K, 1e300, n, N, SEED)
    beta = oracle.cv_beta(o[:, 1], o[:, 2])
    res = mc.mc_price(ctx, model, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, K, cv=mc.MC_CV_GEO_ASIAN),
                      N, n, SEED, mc.Options(prec=mc.MC_FP64, cv_beta=beta))
    y = o[:, 1] - beta * o[:, 2]
    var = float(np.sum((y - y.mean()) ** 2) / (N - 1))
    say(f"  VRF {res['vrf']:.3e}; variance gpu {res['variance']:.12e} oracle {var:.12e}")
    assert res["vrf"] > 1e6
    assert abs(res["variance"] / var - 1.0) < 1e-6
    # A payoff whose variance is 1e-10 of its squared mean (K = 0, sigma =
    # 1e-5): a sum of squares would lose it; the co-moments keep 1e-6.
    model = mc.Model(kind=mc.MC_GBM, S0=S0, r=r_, T=T, sigma=1e-5)
    res = mc.mc_price(ctx, model, mc.Payoff(mc.MC_EURO_CALL, 0.0), N, n, SEED,
                      mc.Options(prec=mc.MC_FP64))
    e = oracle.gbm(S0, r_, 1e-5, T, 0.0, 1e300, n, N, SEED)[:, 0]
    var = float(np.sum((e - e.mean()) ** 2) / (N - 1))
    say(f"  tiny variance: gpu {res['variance']:.12e} oracle {var:.12e}, "
        f"mean^2/var {e.mean() ** 2 / var:.2e}")
    assert e.mean() ** 2 / var > 1e9
    assert abs(res["variance"] / var - 1.0) < 1e-6
