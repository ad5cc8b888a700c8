"""GPU parity of the Longstaff-Schwartz pricer (Sec. II-A.3, Sec. VI-C)
against the FP64 oracle on the same Philox paths.

The exercise decisions compare two floating-point values, so they are
compared as what is unique plus validity: the GPU keeps its path state in
FP32 and the oracle in FP64, so both the stored states and the fitted
continuations differ by rounding (a CPU emulation that only rounds the
oracle's states to FP32 moves the fitted continuations by about 1e-6 and
flips no decision on 2^16 paths). The tests require

* the in-the-money counts and the dates with a regression to agree;
* the fitted continuation values of the two sides, evaluated on the
  oracle's in-the-money states, to agree to 1e-4 of their largest value;
* at most a few paths per 10^4 to change their exercise date, each of them
  borderline at the first date where the two sides decide differently
  (exercise value and continuation within 1e-3 there);
* every other path's cash flow to agree to the FP32 state error, and the
  prices to agree up to what the changed paths account for.

Then degenerate cases (one date, nothing in the money, too few paths for a
regression), determinism, argument errors, and the benchmarked size against
the lattice and the closed-form European max-call.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1906_02818_amd as mc
import synth
from closed_forms import max_call_independent
from lsm_basis import CALL, MAXC, PUT, features, payoff

pytestmark = pytest.mark.gpu
SEED = synth.SEED


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mc.mc_create(0)
    yield c
    c.close()


def setup(d, rho, sig0=0.2):
    S0 = 100.0 + 5.0 * np.arange(d) - 2.5 * (d - 1)
    sigma = sig0 + 0.05 * np.arange(d)
    corr = np.full((d, d), rho) + (1.0 - rho) * np.eye(d)
    kind = mc.MC_GBM if d == 1 else mc.MC_GBM_BASKET
    return S0, sigma, corr, kind


def run_both(ctx, d, rho, kind, K, q, T, M, spd, degree, N, r=0.05, n_oos=0, tag=0, offset=0):
    S0, sigma, corr, mk = setup(d, rho)
    model = mc.Model(kind=mk, S0=S0, r=r, T=T, sigma=sigma, corr=corr if d > 1 else None)
    spec = mc.LsmSpec(payoff=kind, K=K, dividend=q, n_dates=M, steps_per_date=spd,
                      degree=degree, n_paths_oos=n_oos)
    g = mc.mc_price_lsm(ctx, model, spec, N, SEED, mc.Options(stream_tag=tag, path_offset=offset),
                        want_paths=True)
    L = np.linalg.cholesky(corr)
    o = oracle.lsm(S0, sigma, L, r, q, T, kind, K, M, spd, degree, N, SEED, tag=tag,
                   path0=offset, want_paths=True)
    oo = None
    if n_oos:
        oo = oracle.lsm_oos(S0, sigma, L, r, q, T, kind, K, M, spd, degree, o["beta"], n_oos,
                            SEED, tag=tag + 7, path0=offset)
    return g, o, oo


def first_difference(eg, eo, M):
    """Date of the first differing decision: the earlier of the two exercise
    dates (0 = never, read as after t_M)."""
    a = np.where(eg == 0, M + 1, eg)
    b = np.where(eo == 0, M + 1, eo)
    return np.minimum(a, b)


CASES = [
    # d, rho, payoff, K, q, T, M, steps/date, degree, N, first path, tag  (features)
    (2, 0.3, MAXC, 100.0, 0.10, 3.0, 9, 1, 2, (1 << 16) + 77, 0, 0),     # 7
    (1, 0.0, PUT, 100.0, 0.00, 1.0, 10, 4, 3, 50_000, 0, 0),             # 4
    (3, 0.2, MAXC, 100.0, 0.05, 1.0, 6, 2, 2, 40_000, 0, 0),             # 11
    (4, 0.4, PUT, 100.0, 0.00, 1.0, 8, 1, 1, 30_000, 0, 0),              # 5
    (2, 0.0, CALL, 95.0, 0.06, 2.0, 5, 3, 3, 30_011, 0, 0),              # 10
    (2, 0.3, MAXC, 100.0, 0.10, 3.0, 9, 1, 2, 20_000, (1 << 33) + 5, 3),  # offset and tag
    (1, 0.0, PUT, 100.0, 0.00, 1.0, 7, 1, 3, 40_000, 0, 0),              # 4, dates in 4s
    (3, 0.2, MAXC, 100.0, 0.05, 1.0, 6, 1, 2, 30_000, 0, 0),             # 11, dates in 4s
]


@pytest.mark.parametrize("d,rho,kind,K,q,T,M,spd,degree,N,offset,tag", CASES)
def test_lsm_matches_oracle(ctx, d, rho, kind, K, q, T, M, spd, degree, N, offset, tag):
    say("lsm parity", d, rho, kind, K, q, T, M, spd, degree, N, offset, tag)
    r = 0.05
    g, o, oo = run_both(ctx, d, rho, kind, K, q, T, M, spd, degree, N, r=r, n_oos=N, tag=tag,
                        offset=offset)
    nf = o["n_features"]
    assert g["n_features"] == nf
    y = o["y"]
    # In-the-money counts depend on the states alone: only paths on the
    # strike boundary (within FP32 rounding) may differ.
    assert np.abs(g["n_itm"] - o["n_itm"]).max() <= 2
    vo = ~np.isnan(o["beta"][:, 0])
    assert (g["beta_valid"][:M - 1] == vo[:M - 1]).all()
    # Fitted continuations on the oracle's in-the-money states.
    for j in range(1, M):
        if not vo[j - 1]:
            continue
        f = payoff(kind, y[:, j - 1])
        itm = f > 0
        X = features(y[itm, j - 1], f[itm], degree, kind)
        ho, hg = X @ o["beta"][j - 1], X @ g["beta"][j - 1]
        assert np.abs(hg - ho).max() <= 1e-4 * np.abs(ho).max() + 1e-6, j
    # Exercise dates: few changes, each borderline where the sides diverge.
    eg, eo = g["exercise_date"], o["ex"]
    diff = np.nonzero(eg != eo)[0]
    assert diff.size <= max(3, N // 10_000), diff.size
    jd = first_difference(eg, eo, M)
    for p in diff:
        j = jd[p]
        f = payoff(kind, y[p:p + 1, j - 1])[0]
        e = math.exp(-r * T * j / M) * K * f
        h = o["cont"][p, j - 1]
        if j == M or np.isnan(h):
            assert K * f < 1e-3, (p, j, f)      # on the strike boundary
        else:
            assert abs(e - h) < 1e-3 + 1e-5 * abs(h), (p, j, e, h)
    # Cash flows of the paths with the same decisions: FP32 state error.
    same = eg == eo
    Cg, Co = g["cash_flow"], o["C"]
    np.testing.assert_allclose(Cg[same], Co[same], rtol=1e-5, atol=3e-5 * K)
    assert (Cg[eg == 0] == 0).all() and (Cg[eg > 0] > 0).all()
    moved = np.abs(Cg[~same] - Co[~same]).sum() / N
    assert abs(g["price"] - o["price"]) <= moved + 1e-5 * o["price"] + 1e-9
    assert g["price"] == pytest.approx(Cg.mean(), rel=1e-10)
    assert g["european"] == pytest.approx(o["european"], rel=1e-5, abs=1e-7)
    # Out of sample: each side's rule on the same fresh paths.
    ovg, oeg = g["oos_value"], g["oos_exercise_date"]
    ovo, oeo = oo["Y"], oo["ex"]
    dso = oeg != oeo
    assert dso.sum() <= max(3, N // 10_000)
    np.testing.assert_allclose(ovg[~dso], ovo[~dso], rtol=1e-5, atol=3e-5 * K)
    moved = np.abs(ovg[dso] - ovo[dso]).sum() / N
    assert abs(g["price_oos"] - oo["price"]) <= moved + 1e-5 * oo["price"] + 1e-9
    assert g["price_oos"] == pytest.approx(ovg.mean(), rel=1e-10)


def test_single_date_is_the_european_estimate(ctx):
    g, o, _ = run_both(ctx, 2, 0.2, MAXC, 100.0, 0.1, 1.0, 1, 16, 2, 10_000)
    assert g["price"] == g["european"] and g["std_err"] == g["european_se"]
    assert g["price"] == pytest.approx(o["price"], rel=1e-5)
    assert g["n_itm"][0] == o["n_itm"][0]
    assert set(np.unique(g["exercise_date"])) <= {0, 1}


def test_nothing_in_the_money_prices_zero(ctx):
    g, _, _ = run_both(ctx, 1, 0.0, CALL, 1e6, 0.0, 1.0, 6, 1, 2, 4096)
    assert g["price"] == 0.0 and g["std_err"] == 0.0
    assert (g["beta_valid"] == 0).all() and (g["n_itm"] == 0).all()
    assert (g["exercise_date"] == 0).all()


def test_too_few_paths_skip_the_same_dates(ctx):
    g, o, _ = run_both(ctx, 2, 0.0, MAXC, 125.0, 0.1, 3.0, 9, 1, 2, 16)
    skipped = o["n_itm"][:-1] < o["n_features"]
    assert skipped.any()
    assert (g["n_itm"] == o["n_itm"]).all()
    assert (g["beta_valid"][:-1] == ~np.isnan(o["beta"][:-1, 0])).all()
    assert (g["exercise_date"] == o["ex"]).all()


def test_runs_are_deterministic(ctx):
    S0, sigma, corr, mk = setup(2, 0.3)
    model = mc.Model(kind=mk, S0=S0, r=0.05, T=3.0, sigma=sigma, corr=corr)
    spec = mc.LsmSpec(payoff=MAXC, K=100.0, dividend=0.1, n_dates=9, degree=2,
                      n_paths_oos=1 << 18)
    a = mc.mc_price_lsm(ctx, model, spec, (1 << 20) + 3, SEED, want_paths=True)
    b = mc.mc_price_lsm(ctx, model, spec, (1 << 20) + 3, SEED, want_paths=True)
    for k in ("price", "std_err", "price_oos", "european"):
        assert a[k] == b[k], k
    assert np.array_equal(a["cash_flow"], b["cash_flow"])
    assert np.array_equal(a["beta"], b["beta"], equal_nan=True)


def test_benchmarked_size_against_lattice_and_closed_form(ctx):
    # The two-asset max-call of the benchmark, 2^24 paths in and out of sample.
    say("lsm full size")
    S0, sigma = np.array([100.0, 100.0]), np.array([0.2, 0.2])
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=S0, r=0.05, T=3.0, sigma=sigma, corr=np.eye(2))
    spec = mc.LsmSpec(payoff=MAXC, K=100.0, dividend=0.1, n_dates=9, steps_per_date=1,
                      degree=2, n_paths_oos=1 << 24)
    g = mc.mc_price_lsm(ctx, model, spec, 1 << 24, SEED)
    true = oracle.lsm_lattice(S0, sigma, 0.05, 0.1, 3.0, MAXC, 100.0, 9, 50)
    euro = max_call_independent(S0, sigma, 0.05, 0.1, 3.0, 100.0)
    assert abs(g["european"] - euro) < 4 * g["european_se"]
    assert abs(g["price"] - true) < 3 * g["std_err"] + 0.01 * true
    assert g["price_oos"] < true + 3 * g["std_err_oos"]
    assert g["price_oos"] > true - 3 * g["std_err_oos"] - 0.01 * true
    assert g["beta_valid"][:8].all()


def test_argument_errors(ctx):
    S0, sigma, corr, mk = setup(2, 0.3)
    good = dict(kind=mk, S0=S0, r=0.05, T=1.0, sigma=sigma, corr=corr)
    spec = dict(payoff=MAXC, K=100.0, dividend=0.0, n_dates=4, steps_per_date=1, degree=2)

    def status(model=None, n=1000, opts=None, **kw):
        m = mc.Model(**(model or good))
        s = mc.LsmSpec(**{**spec, **kw})
        with pytest.raises(mc.McError) as e:
            mc.mc_price_lsm(ctx, m, s, n, SEED, opts)
        return str(e.value)

    assert "INVALID_ARG" in status(payoff=0)
    assert "INVALID_ARG" in status(K=0.0)
    assert "INVALID_ARG" in status(dividend=float("nan"))
    assert "INVALID_ARG" in status(n_dates=0)
    assert "INVALID_ARG" in status(n_dates=65)
    assert "INVALID_ARG" in status(steps_per_date=0)
    assert "INVALID_ARG" in status(degree=0)
    assert "INVALID_ARG" in status(degree=4)
    assert "INVALID_ARG" in status(n=1)
    assert "INVALID_ARG" in status(n_paths_oos=1)
    five = dict(good, S0=np.full(5, 100.0), sigma=np.full(5, 0.2), corr=np.eye(5))
    assert "INVALID_ARG" in status(model=five)
    three = dict(good, S0=np.full(3, 100.0), sigma=np.full(3, 0.2), corr=np.eye(3))
    assert "UNSUPPORTED" in status(model=three, degree=3)
    assert "UNSUPPORTED" in status(opts=mc.Options(prec=mc.MC_BF16_GEMM))
    assert "UNSUPPORTED" in status(opts=mc.Options(greeks=mc.MC_GREEK_DELTA))
    bad = dict(good, corr=np.array([[1.0, 1.2], [1.2, 1.0]]))
    assert "NOT_PD" in status(model=bad)
    heston = dict(kind=mc.MC_HESTON, S0=[100.0], r=0.05, T=1.0, v0=0.04, kappa=1.0,
                  theta=0.04, xi=0.5, rho=-0.5)
    assert "UNSUPPORTED" in status(model=heston)
