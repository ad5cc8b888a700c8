"""FP64 CPU oracle for the Monte Carlo path engine -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product library never loads it and
shares no code with it.

The arithmetic lives in ``mc_oracle.c`` (plain double precision, one path and
one step at a time). This module only marshals numpy arrays through ctypes
and adds the estimator formulas of Eq. (3) and the bias-variance split of
Sec. V-B, plus the Adam update used to train the learned control variate.

The arithmetic-Asian call price has no closed form for many fixings; the
tests pin its K = 0 mean, its zero-volatility value at any K, its ordering
against the geometric Asian, its pathwise tangents, its one-fixing case (the
European call) and its two-fixing price at K > 0 with volatility (a
one-dimensional quadrature of a Black-Scholes inner expectation).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")

GBM_CHANNELS = ("euro", "asian", "geo", "uo", "euro_delta", "euro_vega",
                "asian_delta", "asian_vega", "disc_ST", "uo_bridge", "uo_margin",
                "uo_bridge_margin")
HESTON_CHANNELS = ("euro", "asian", "euro_delta", "euro_dv0", "asian_delta",
                   "asian_dv0", "disc_ST")
BASKET_CHANNELS = ("basket", "geo_basket", "delta0")
MLP_NPARAM = 4545


def lib():
    """Loads liboracle.so (built by oracle/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: run oracle/build.py")
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_normal.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64]
        L.orc_normal.restype = C.c_double
        L.orc_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64,
                                  C.c_uint64, _dp]
        L.orc_words_many.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, _u64p,
                                     _u64p, _u32p]
        L.orc_gbm.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_uint64,
                              C.c_uint32, C.c_uint64, C.c_uint64, _dp]
        L.orc_gbm_payoffs.argtypes = L.orc_gbm.argtypes
        L.orc_heston.argtypes = [_dp, C.c_int, C.c_uint64, C.c_uint32, C.c_uint64,
                                 C.c_uint64, _dp]
        L.orc_cholesky.argtypes = [C.c_int, _dp, _dp]
        L.orc_cholesky.restype = C.c_int
        L.orc_basket.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_double,
                                 C.c_double, C.c_double, C.c_int, C.c_uint64,
                                 C.c_uint32, C.c_uint64, C.c_uint64, _dp]
        L.orc_bs_call.argtypes = [C.c_double] * 5
        L.orc_bs_call.restype = C.c_double
        L.orc_portfolio_premium.argtypes = [C.c_int, _dp, _dp, C.c_int, _dp, _dp,
                                            C.c_double, C.c_double]
        L.orc_portfolio_premium.restype = C.c_double
        L.orc_portfolio_pnl.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_int, _dp, _dp,
                                        C.c_double, C.c_double, C.c_int, C.c_uint64,
                                        C.c_uint32, C.c_uint64, C.c_uint64, _dp]
        L.orc_sobol_polys.argtypes = [C.c_int, np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS"),
                                      _u32p]
        L.orc_sobol_polys.restype = C.c_int
        L.orc_sobol_dirs.argtypes = [C.c_int, _u32p]
        L.orc_sobol_word.argtypes = [_u32p, C.c_int, C.c_uint64]
        L.orc_sobol_word.restype = C.c_uint32
        L.orc_qmc_shifts.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int, _u32p]
        L.orc_basket_qmc.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_double, C.c_double,
                                     C.c_double, C.c_int, C.c_uint64, C.c_uint32, C.c_uint64,
                                     C.c_uint64, C.c_uint64, _dp]
        _i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        L.orc_lsm_n_features.argtypes = [C.c_int, C.c_int, C.c_int]
        L.orc_lsm_n_features.restype = C.c_int
        L.orc_lsm.argtypes = [C.c_int, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                              C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.c_uint64,
                              C.c_uint32, C.c_uint64, C.c_uint64, _dp, _dp, _i64p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_lsm.restype = C.c_int
        L.orc_lsm_oos.argtypes = [C.c_int, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                  C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, _dp,
                                  C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, _dp,
                                  C.c_void_p, C.c_void_p]
        L.orc_lsm_oos.restype = C.c_int
        L.orc_lsm_lattice.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                      C.c_int, C.c_double, C.c_int, C.c_int]
        L.orc_lsm_lattice.restype = C.c_double
        L.orc_heston_cv.argtypes = [_dp, C.c_int, C.c_int, _dp, C.c_uint64,
                                    C.c_uint32, C.c_uint64, C.c_uint64, C.c_int, _dp]
        L.orc_mlp_eval.argtypes = [_dp, C.c_uint64, _dp, C.c_int, _dp]
        L.orc_bf16_round.argtypes = [C.c_double]
        L.orc_bf16_round.restype = C.c_double
        L.orc_cv_loss_grad.argtypes = [_dp, C.c_int, C.c_int, _dp, C.c_uint64,
                                       C.c_uint32, C.c_uint64, C.c_uint64, C.c_void_p]
        L.orc_cv_loss_grad.restype = C.c_double
        for f in ("orc_gbm_channels", "orc_heston_channels", "orc_basket_channels",
                  "orc_mlp_nparam"):
            getattr(L, f).restype = C.c_int
        assert L.orc_gbm_channels() == len(GBM_CHANNELS)
        assert L.orc_heston_channels() == len(HESTON_CHANNELS)
        assert L.orc_basket_channels() == len(BASKET_CHANNELS)
        assert L.orc_mlp_nparam() == MLP_NPARAM
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# Random numbers (Sec. IV-A): Philox4x32-10 block function, counter layout,
# open-interval uniform and Box-Muller.
# --------------------------------------------------------------------------
def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.ascontiguousarray(ctr, np.uint32),
                            np.ascontiguousarray(key, np.uint32), out)
    return out


def words(seed: int, tag: int, paths, blocks) -> np.ndarray:
    paths = np.ascontiguousarray(paths, np.uint64)
    blocks = np.ascontiguousarray(blocks, np.uint64)
    out = np.zeros((paths.size, 4), np.uint32)
    lib().orc_words_many(seed, tag, paths.size, paths, blocks, out)
    return out


def uniform(w: int) -> float:
    return lib().orc_uniform(int(w))


def normal(seed: int, tag: int, path: int, k: int) -> float:
    return lib().orc_normal(seed, tag, path, k)


def normals(seed: int, tag: int, path: int, k0: int, count: int) -> np.ndarray:
    out = np.zeros(count, np.float64)
    lib().orc_normals(seed, tag, path, k0, count, out)
    return out


# --------------------------------------------------------------------------
# Path simulators: per-path channel rows.
# --------------------------------------------------------------------------
def gbm(S0, r, sigma, T, K, B, n_steps, n_paths, seed, tag=0, path0=0,
        scheme=0, coarsen=1, payoffs_only=False) -> np.ndarray:
    """Per-path GBM channels; payoffs_only computes channels 0-3 and 8 only
    (the others NaN): no tangents, Brownian-bridge stream or margins."""
    prm = np.array([S0, r, sigma, T, K, B], np.float64)
    out = np.zeros((n_paths, len(GBM_CHANNELS)), np.float64)
    fn = lib().orc_gbm_payoffs if payoffs_only else lib().orc_gbm
    fn(prm, n_steps, scheme, coarsen, seed, tag, path0, n_paths, out)
    return out


def heston(S0, v0, kappa, theta, xi, rho, r, T, K, n_steps, n_paths, seed,
           tag=0, path0=0) -> np.ndarray:
    prm = np.array([S0, v0, kappa, theta, xi, rho, r, T, K], np.float64)
    out = np.zeros((n_paths, len(HESTON_CHANNELS)), np.float64)
    lib().orc_heston(prm, n_steps, seed, tag, path0, n_paths, out)
    return out


def cholesky(Cm: np.ndarray) -> np.ndarray | None:
    Cm = np.ascontiguousarray(Cm, np.float64)
    d = Cm.shape[0]
    L = np.zeros((d, d), np.float64)
    st = lib().orc_cholesky(d, Cm, L)
    return None if st != 0 else L


def basket(S0, sigma, L, w, r, T, K, n_steps, n_paths, seed, tag=0,
           path0=0) -> np.ndarray:
    S0 = np.ascontiguousarray(S0, np.float64)
    sigma = np.ascontiguousarray(sigma, np.float64)
    L = np.ascontiguousarray(L, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    d = S0.size
    out = np.zeros((n_paths, len(BASKET_CHANNELS)), np.float64)
    lib().orc_basket(d, S0, sigma, L, w, r, T, K, n_steps, seed, tag, path0,
                     n_paths, out)
    return out


def portfolio_premium(S0, sigma, m, q, r, T) -> float:
    """Black-Scholes value at time 0 of q_k calls of strike m_k S0_a on every
    asset (Sec. VI-B.1 portfolio)."""
    S0, sigma = _c(S0), _c(sigma)
    m, q = _c(m), _c(q)
    return lib().orc_portfolio_premium(S0.size, S0, sigma, m.size, m, q, r, T)


def portfolio_pnl(S0, sigma, mu, L, m, q, r, T, n_steps, n_paths, seed, tag=0,
                  path0=0) -> np.ndarray:
    """Per-path horizon P&L of the call portfolio on d correlated GBM assets
    with real-world drifts mu (Sec. VI-B.1)."""
    S0, sigma, mu, L = _c(S0), _c(sigma), _c(mu), _c(L)
    m, q = _c(m), _c(q)
    out = np.zeros(n_paths, np.float64)
    lib().orc_portfolio_pnl(S0.size, S0, sigma, mu, L, m.size, m, q, r, T, n_steps,
                            seed, tag, path0, n_paths, out)
    return out


def var_cvar(pnl, alpha):
    """Empirical Value-at-Risk and Conditional Value-at-Risk of Sec. VI-B.1.
    VaR_alpha = -inf{x : F_N(x) > 1 - alpha}, the k-th smallest P&L with
    k = floor(N (1 - alpha)) + 1; CVaR_alpha = -mean{PnL_i : -PnL_i > VaR}.
    Returns (VaR, CVaR, k, number of tail paths)."""
    x = np.sort(np.asarray(pnl, np.float64))
    N = x.size
    k = int(np.floor(N * (1.0 - alpha))) + 1
    var = -x[k - 1]
    tail = x[x < x[k - 1]]
    cvar = -tail.mean() if tail.size else float("nan")
    return var, cvar, k, tail.size


def sobol_polys(n):
    """First n primitive polynomials over GF(2) (degree, bit pattern)."""
    deg = np.zeros(n, np.int32)
    poly = np.zeros(n, np.uint32)
    k = lib().orc_sobol_polys(n, deg, poly)
    return deg[:k], poly[:k]


def sobol_dirs(n_dims) -> np.ndarray:
    """Direction words V[dim, bit] of the Sobol' construction (section 11)."""
    V = np.zeros((n_dims, 32), np.uint32)
    lib().orc_sobol_dirs(n_dims, V.reshape(-1))
    return V


def sobol_points(V, n_points, point0=0) -> np.ndarray:
    """Unshifted 32-bit coordinates [n_points, n_dims]."""
    n_dims = V.shape[0]
    Vf = np.ascontiguousarray(V.reshape(-1))
    out = np.zeros((n_points, n_dims), np.uint32)
    for i in range(n_points):
        for j in range(n_dims):
            out[i, j] = lib().orc_sobol_word(Vf, j, point0 + i)
    return out


def qmc_shifts(seed, tag, replicate, n_dims) -> np.ndarray:
    sh = np.zeros(n_dims, np.uint32)
    lib().orc_qmc_shifts(seed, tag, replicate, n_dims, sh)
    return sh


def basket_qmc(S0, sigma, L, w, r, T, K, n_steps, n_paths, seed, replicate, tag=6,
               path0=0) -> np.ndarray:
    """Basket channels on Sobol' points with the digital shift of `replicate`."""
    S0, sigma, L, w = _c(S0), _c(sigma), _c(L), _c(w)
    out = np.zeros((n_paths, len(BASKET_CHANNELS)), np.float64)
    lib().orc_basket_qmc(S0.size, S0, sigma, L, w, r, T, K, n_steps, seed, tag, replicate,
                         path0, n_paths, out)
    return out


# --------------------------------------------------------------------------
# Longstaff-Schwartz regression for Bermudan options (Sec. II-A.3, VI-C) and
# the binomial lattice that gives the value it estimates.
# --------------------------------------------------------------------------
LSM_MAX_CALL, LSM_BASKET_PUT, LSM_BASKET_CALL = 1, 2, 3


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def lsm_n_features(d, degree, kind) -> int:
    return lib().orc_lsm_n_features(d, degree, kind)


def lsm(S0, sigma, L, r, q, T, kind, K, n_dates, steps_per_date, degree, n_paths, seed,
        tag=0, path0=0, want_paths=False) -> dict:
    """In-sample Longstaff-Schwartz estimate and everything it decided."""
    S0, sigma, L = _c(S0), _c(sigma), _c(L)
    d, M, n = S0.size, n_dates, n_paths
    nf = lsm_n_features(d, degree, kind)
    res = np.zeros(4)
    beta = np.zeros((M, nf))
    n_itm = np.zeros(M, np.int64)
    Cf = np.zeros(n)
    ex = np.zeros(n, np.int32)
    cont = np.zeros((n, M))
    y = np.zeros((n, M, d)) if want_paths else None
    got = lib().orc_lsm(d, S0, sigma, L, r, q, T, kind, K, M, steps_per_date, degree, seed,
                        tag, path0, n, res, beta, n_itm, _ptr(Cf), _ptr(ex), _ptr(cont), _ptr(y))
    if got != nf:
        raise ValueError("orc_lsm rejected its arguments")
    out = {"price": res[0], "std_err": res[1], "european": res[2], "european_se": res[3],
           "beta": beta, "n_itm": n_itm, "C": Cf, "ex": ex, "cont": cont, "n_features": nf}
    if want_paths:
        out["y"] = y
    return out


def lsm_oos(S0, sigma, L, r, q, T, kind, K, n_dates, steps_per_date, degree, beta, n_paths,
            seed, tag=7, path0=0) -> dict:
    """Out-of-sample estimate: the exercise rule of `beta` on fresh paths."""
    S0, sigma, L = _c(S0), _c(sigma), _c(L)
    res = np.zeros(2)
    Y = np.zeros(n_paths)
    ex = np.zeros(n_paths, np.int32)
    got = lib().orc_lsm_oos(S0.size, S0, sigma, L, r, q, T, kind, K, n_dates, steps_per_date,
                            degree, _c(beta), seed, tag, path0, n_paths, res, _ptr(Y), _ptr(ex))
    if got < 0:
        raise ValueError("orc_lsm_oos rejected its arguments")
    return {"price": res[0], "std_err": res[1], "Y": Y, "ex": ex}


def lsm_lattice(S0, sigma, r, q, T, kind, K, n_dates, tree_steps_per_date) -> float:
    S0, sigma = _c(S0), _c(sigma)
    v = lib().orc_lsm_lattice(S0.size, S0, sigma, r, q, T, kind, K, n_dates,
                              tree_steps_per_date)
    if v < 0:
        raise ValueError("orc_lsm_lattice rejected its arguments")
    return v


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(np.atleast_1d(np.asarray(a, np.float64)))


def _heston_prm(h: dict) -> np.ndarray:
    return np.array([h["S0"], h["v0"], h["kappa"], h["theta"], h["xi"],
                     h["rho"], h["r"], h["T"], h["K"]], np.float64)


def heston_cv(h: dict, n_steps, theta, n_paths, seed, tag=0, path0=0,
              m_every=1, bf16=False) -> np.ndarray:
    """Per-path (discounted Asian payoff, hedge P&L H, payoff - H); bf16
    rounds the operands of the network's two matrix products to bfloat16."""
    out = np.zeros((n_paths, 3), np.float64)
    lib().orc_heston_cv(_heston_prm(h), n_steps, m_every,
                        np.ascontiguousarray(theta, np.float64), seed, tag,
                        path0, n_paths, int(bf16), out)
    return out


def mlp_eval(theta, phi, bf16=False) -> np.ndarray:
    phi = np.ascontiguousarray(phi, np.float64).reshape(-1, 4)
    out = np.zeros(phi.shape[0], np.float64)
    lib().orc_mlp_eval(np.ascontiguousarray(theta, np.float64), phi.shape[0],
                       phi, int(bf16), out)
    return out


def bf16_round(x: float) -> float:
    return lib().orc_bf16_round(float(x))


def cv_loss_grad(h: dict, n_steps, theta, B, seed, tag=2, path0=0,
                 m_every=1, want_grad=True):
    grad = np.zeros(MLP_NPARAM, np.float64) if want_grad else None
    loss = lib().orc_cv_loss_grad(
        _heston_prm(h), n_steps, m_every,
        np.ascontiguousarray(theta, np.float64), seed, tag, path0, B,
        grad.ctypes.data if want_grad else None)
    return loss, grad


# --------------------------------------------------------------------------
# Estimators (Eq. 3; standard error from the variance term of Sec. V-B,
# read as Var(f(X))/N).
# --------------------------------------------------------------------------
def estimate(y: np.ndarray) -> dict:
    y = np.asarray(y, np.float64)
    n = y.size
    mean = float(np.sum(y) / n)
    var = float(np.sum((y - mean) ** 2) / (n - 1))
    return {"price": mean, "variance": var, "std_err": float(np.sqrt(var / n)),
            "n": n}


def cv_beta(a: np.ndarray, g: np.ndarray) -> float:
    """Least-squares control-variate coefficient cov(a,g)/var(g)."""
    a = np.asarray(a, np.float64)
    g = np.asarray(g, np.float64)
    am, gm = a.mean(), g.mean()
    return float(np.sum((a - am) * (g - gm)) / np.sum((g - gm) ** 2))


def cv_estimate(a: np.ndarray, g: np.ndarray, g_mean: float, beta: float) -> dict:
    """Estimate of E[a] through Y = a - beta (g - E[g])."""
    return estimate(np.asarray(a) - beta * (np.asarray(g) - g_mean))


# --------------------------------------------------------------------------
# Adam (Kingma and Ba, 2015), the optimiser of the learned control variate.
# --------------------------------------------------------------------------
def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One update at step t >= 1; returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
