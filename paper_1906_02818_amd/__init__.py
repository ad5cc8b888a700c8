"""MI355X (gfx950) Monte Carlo path engine: Python binding of include/mcpath.h.

Every function here marshals arguments into the C ABI of libmcpath.so and
returns its outputs; all path simulation, payoff evaluation and reduction
runs in the library's HIP kernels. PyTorch supplies the device workspace and
the stream when a GPU is visible. If the library is missing, every call
raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass, field, replace
from typing import Sequence

import numpy as np

from . import _abi
from ._abi import (MC_ADJ_FULL, MC_ADJ_FWD, MC_ADJ_REV, MC_ASIAN_ARITH_CALL, MC_ASIAN_GEO_CALL,
                   MC_BASKET_CALL, MC_BF16X2_GEMM, MC_BF16_GEMM, MC_COUPLE_NONE,
                   MC_COUPLE_PRECISION, MC_COUPLE_TIME, MC_CV_GEO_ASIAN, MC_CV_LEARNED,
                   MC_CV_NONE, MC_ERR_DEVICE, MC_ERR_INVALID_ARG, MC_ERR_NOT_PD, MC_ERR_NO_DEVICE,
                   MC_ERR_OOM, MC_ERR_UNSUPPORTED, MC_ERR_WORKSPACE, MC_EULER_S, MC_EURO_CALL,
                   MC_FP16_GEMM, MC_FP32, MC_FP64, MC_GBM, MC_GBM_BASKET, MC_GREEKS_FD_CRN,
                   MC_GREEKS_PATHWISE, MC_GREEKS_TANGENT, MC_GREEK_DELTA, MC_GREEK_VEGA,
                   MC_HESTON, MC_LOG_EULER, MC_LSM_BASKET_CALL, MC_LSM_BASKET_PUT,
                   MC_LSM_MAX_CALL, MC_LSM_MAX_DATES, MC_LSM_MAX_FEATURES, MC_MAX_STRIKES, MC_MLMC_MAX_LEVELS, MC_MLP_NPARAM, MC_OK,
                   MC_PILOT_IN_SAMPLE,
                   MC_QMC_MAX_REPLICATES, MC_UO_BARRIER_CALL, MC_UO_BRIDGE_CALL)

__all__ = [n for n in dir(_abi) if n.startswith("MC_")] + [
    "McError", "Model", "Payoff", "Options", "mc_create", "mc_destroy", "mc_validate",
    "mc_price", "mc_price_multi", "mc_greeks_adjoint", "mc_cv_train", "mc_cv_loss_grad",
    "mc_philox_words", "mc_normals", "mc_path_channels", "mc_path_channel_name",
    "mc_workspace_bytes", "mc_adjoint_ckpt_bytes", "mc_status_str", "mc_last_error",
    "mc_price_mlmc", "mc_mlmc_allocate", "Level", "mc_risk", "mc_price_qmc", "PathwisePrice", "TangentPrice",
    "LsmSpec", "mc_price_lsm",
    "PreparedPriceMulti"]


class McError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{mc_status_str(status)}: {message}")
        self.status = status


@dataclass
class Model:
    kind: int = MC_GBM
    S0: Sequence[float] | float = 100.0
    r: float = 0.0
    T: float = 1.0
    sigma: Sequence[float] | float | None = None
    corr: np.ndarray | None = None
    v0: float = 0.0
    kappa: float = 0.0
    theta: float = 0.0
    xi: float = 0.0
    rho: float = 0.0
    scheme: int = MC_LOG_EULER


@dataclass
class Payoff:
    kind: int = MC_EURO_CALL
    K: float = 100.0
    B: float = math.inf
    weights: Sequence[float] | None = None
    cv: int = MC_CV_NONE


@dataclass
class Options:
    prec: int = MC_FP32
    greeks: int = 0
    path_offset: int = 0
    stream_tag: int = 0
    cv_weights: np.ndarray | None = None
    cv_hedge_every: int = 1
    cv_beta: float = math.nan
    pilot_paths: int = 0
    path_values: bool = False      # also return per-path channel values
    greeks_method: int = MC_GREEKS_PATHWISE
    fd_rel_step: float = 1e-3


def _arr(x, dtype=np.float64):
    return np.ascontiguousarray(np.atleast_1d(np.asarray(x, dtype=dtype)))


class _Marshal:
    """Keeps the numpy buffers alive while a C call runs."""

    def __init__(self, model: Model, payoff: Payoff | Sequence[Payoff], opts: Options | None,
                 n_paths: int, torch_ws: bool = True):
        self.keep = []
        self.cm = self._model(model)
        if isinstance(payoff, Payoff):
            self.cp = self._payoff(payoff)
            self.cps = None
        else:
            self.cps = (_abi.McPayoff * len(payoff))(*[self._payoff(p) for p in payoff])
            self.cp = self.cps[0]
        self.opts = opts or Options()
        self.co = self._options(self.opts)
        self.path_buf = None

    def _ptr(self, a, ctype):
        self.keep.append(a)
        return a.ctypes.data_as(C.POINTER(ctype))

    def _model(self, m: Model):
        S0 = _arr(m.S0)
        cm = _abi.McModel()
        cm.kind = m.kind
        cm.dim = S0.size
        cm.r = m.r
        cm.T = m.T
        cm.S0 = self._ptr(S0, C.c_double)
        if m.sigma is not None:
            cm.sigma = self._ptr(_arr(m.sigma), C.c_double)
        if m.corr is not None:
            cm.corr = self._ptr(_arr(np.asarray(m.corr, np.float64).ravel()), C.c_double)
        cm.v0, cm.kappa, cm.theta, cm.xi, cm.rho = m.v0, m.kappa, m.theta, m.xi, m.rho
        cm.scheme = m.scheme
        return cm

    def _payoff(self, f: Payoff):
        cp = _abi.McPayoff()
        cp.kind = f.kind
        cp.K = f.K
        cp.B = f.B
        if f.weights is not None:
            cp.weights = self._ptr(_arr(f.weights), C.c_double)
        cp.cv = f.cv
        return cp

    def _options(self, o: Options):
        co = _abi.McOptions()
        _abi.load().mc_options_default(C.byref(co))
        co.prec = o.prec
        co.greeks = o.greeks
        co.path_offset = o.path_offset
        co.stream_tag = o.stream_tag
        if o.cv_weights is not None:
            w = np.ascontiguousarray(o.cv_weights, np.float32)
            if w.size != MC_MLP_NPARAM:
                raise ValueError(f"cv_weights needs {MC_MLP_NPARAM} values")
            co.cv_weights = self._ptr(w, C.c_float)
        co.cv_hedge_every = o.cv_hedge_every
        co.cv_beta = o.cv_beta
        co.pilot_paths = o.pilot_paths
        co.greeks_method = o.greeks_method
        co.fd_rel_step = o.fd_rel_step
        return co

    def want_path_values(self, n_paths: int, n_channels: int):
        self.path_buf = np.zeros((n_paths, n_channels), np.float64)
        self.co.path_values = self._ptr(self.path_buf, C.c_double)

    def attach_torch(self, ctx: "Context", n_paths: int, n_steps: int):
        """Workspace and stream from PyTorch's caching allocator / current stream."""
        torch = _torch()
        if torch is None:
            return
        need = _abi.load().mc_workspace_bytes(C.byref(self.cm), C.byref(self.cp), n_paths,
                                              n_steps, C.byref(self.co))
        if need == 0:
            return
        ws = ctx.workspace(need)
        self.co.workspace = ws.data_ptr()
        self.co.workspace_bytes = ws.numel()
        self.co.hip_stream = torch.cuda.current_stream(ctx.device).cuda_stream


def _torch():
    try:
        import torch
    except Exception:  # pragma: no cover
        return None
    if not torch.cuda.is_available():
        return None
    return torch


def _check(ctx, st):
    if st != MC_OK:
        msg = _abi.load().mc_last_error(ctx.handle if ctx else None)
        raise McError(st, msg.decode() if msg else "")


def _result(r: _abi.McResult) -> dict:
    return {name: getattr(r, name) for name, _ in _abi.McResult._fields_}


class Context:
    """Owns an mc_context; caches a torch workspace tensor."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        st = _abi.load().mc_create(C.byref(h), device)
        if st != MC_OK:
            raise McError(st, f"mc_create(device={device})")
        self.handle = h
        self.device = device
        self._ws = None

    def workspace(self, nbytes: int):
        torch = _torch()
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def close(self):
        if self.handle:
            _abi.load().mc_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------- C ABI names --
def mc_create(device: int = 0) -> Context:
    return Context(device)


def mc_destroy(ctx: Context) -> None:
    ctx.close()


def mc_status_str(st: int) -> str:
    return _abi.load().mc_status_str(st).decode()


def mc_last_error(ctx: Context | None) -> str:
    return _abi.load().mc_last_error(ctx.handle if ctx else None).decode()


def mc_validate(model: Model, payoff: Payoff, n_paths: int, n_steps: int,
                opts: Options | None = None) -> int:
    """Returns the mc_status of the argument checks (no device needed)."""
    mm = _Marshal(model, payoff, opts, n_paths)
    return _abi.load().mc_validate(None, C.byref(mm.cm), C.byref(mm.cp), n_paths, n_steps,
                                   C.byref(mm.co))


def mc_path_channels(model: Model, payoff: Payoff, opts: Options | None = None) -> list[str]:
    mm = _Marshal(model, payoff, opts, 2)
    lib = _abi.load()
    n = lib.mc_path_channels(C.byref(mm.cm), C.byref(mm.cp), C.byref(mm.co))
    return [lib.mc_path_channel_name(C.byref(mm.cm), C.byref(mm.cp), C.byref(mm.co), i).decode()
            for i in range(n)]


def mc_path_channel_name(model: Model, payoff: Payoff, opts: Options | None, i: int) -> str:
    return mc_path_channels(model, payoff, opts)[i]


def mc_workspace_bytes(model: Model, payoff: Payoff, n_paths: int, n_steps: int,
                       opts: Options | None = None) -> int:
    mm = _Marshal(model, payoff, opts, n_paths)
    return _abi.load().mc_workspace_bytes(C.byref(mm.cm), C.byref(mm.cp), n_paths, n_steps,
                                          C.byref(mm.co))


def mc_adjoint_ckpt_bytes(n_paths: int, n_steps: int, ckpt_every: int = 16) -> int:
    return _abi.load().mc_adjoint_ckpt_bytes(n_paths, n_steps, ckpt_every)


def mc_price(ctx: Context, model: Model, payoff: Payoff, n_paths: int, n_steps: int, seed: int,
             opts: Options | None = None) -> dict:
    mm = _Marshal(model, payoff, opts, n_paths)
    if mm.opts.path_values:
        names = mc_path_channels(model, payoff, opts)
        mm.want_path_values(n_paths, len(names))
    mm.attach_torch(ctx, n_paths, n_steps)
    res = _abi.McResult()
    st = _abi.load().mc_price(ctx.handle, C.byref(mm.cm), C.byref(mm.cp), n_paths, n_steps, seed,
                              C.byref(mm.co), C.byref(res))
    _check(ctx, st)
    out = _result(res)
    if mm.path_buf is not None:
        out["path_values"] = mm.path_buf
        out["path_channels"] = names
    return out


def mc_noalloc_scratch_bytes() -> int:
    return _abi.load().mc_noalloc_scratch_bytes()


def mc_price_noalloc(ctx: Context, model: Model, payoff: Payoff, n_paths: int, n_steps: int,
                     seed: int, opts: Options | None = None) -> dict:
    """mc_price without device allocation: the library's static per-GPU
    scratch holds the run's moments; no workspace tensor is attached."""
    mm = _Marshal(model, payoff, opts, n_paths)
    if mm.opts.path_values:      # passed through so that the library refuses it
        mm.want_path_values(n_paths, max(1, len(mc_path_channels(model, payoff, opts))))
    res = _abi.McResult()
    st = _abi.load().mc_price_noalloc(ctx.handle, C.byref(mm.cm), C.byref(mm.cp), n_paths,
                                      n_steps, seed, C.byref(mm.co), C.byref(res))
    _check(ctx, st)
    return _result(res)


def mc_price_multi(ctx: Context, model: Model, payoffs: Sequence[Payoff], n_paths: int,
                   n_steps: int, seed: int, opts: Options | None = None) -> list[dict]:
    mm = _Marshal(model, list(payoffs), opts, n_paths)
    res = (_abi.McResult * len(payoffs))()
    st = _abi.load().mc_price_multi(ctx.handle, C.byref(mm.cm), mm.cps, len(payoffs), n_paths,
                                    n_steps, seed, C.byref(mm.co), res)
    _check(ctx, st)
    return [_result(r) for r in res]


@dataclass
class Level:
    """One level of a multilevel estimate (mc_level)."""
    n_steps: int
    prec: int
    n_paths: int


def mc_price_mlmc(ctx: Context, model: Model, payoff: Payoff, levels: Sequence[Level], seed: int,
                  opts: Options | None = None) -> dict:
    """Multilevel estimate: level 0 plain, level l the correction P_l - P_{l-1}
    on paths shared by both configurations (mc_price_mlmc)."""
    mm = _Marshal(model, payoff, opts, max(lv.n_paths for lv in levels))
    torch = _torch()
    if torch is not None:
        mm.co.hip_stream = torch.cuda.current_stream(ctx.device).cuda_stream
    arr = (_abi.McLevel * len(levels))(
        *[_abi.McLevel(int(lv.n_steps), int(lv.prec), int(lv.n_paths)) for lv in levels])
    res = _abi.McMlmcResult()
    st = _abi.load().mc_price_mlmc(ctx.handle, C.byref(mm.cm), C.byref(mm.cp), len(levels), arr,
                                   seed, C.byref(mm.co), C.byref(res))
    _check(ctx, st)
    n = res.n_levels
    lv = [{k: getattr(res, k)[i] for k in ("coupling", "mean", "variance", "fine_mean",
                                           "coarse_mean", "n_paths", "kernel_ms")}
          for i in range(n)]
    return {"price": res.price, "std_err": res.std_err, "levels": lv}


def mc_mlmc_allocate(var: Sequence[float], cost: Sequence[float], target_se: float) -> list[int]:
    """Cost-optimal path counts per level for a target standard error."""
    v = _arr(var)
    c = _arr(cost)
    if v.size != c.size:
        raise ValueError("var and cost differ in length")
    out = np.zeros(v.size, np.uint64)
    st = _abi.load().mc_mlmc_allocate(v.size, v.ctypes.data_as(C.POINTER(C.c_double)),
                                      c.ctypes.data_as(C.POINTER(C.c_double)), float(target_se),
                                      out.ctypes.data_as(C.POINTER(C.c_uint64)))
    _check(None, st)
    return [int(x) for x in out]


def mc_risk(ctx: Context, model: Model, strike_mult: Sequence[float], quantity: Sequence[float],
            alpha: float, n_paths: int, n_steps: int, seed: int, mu=None,
            opts: Options | None = None) -> dict:
    """Horizon P&L of a call portfolio on the basket's assets under drifts mu
    (None: the model's r); VaR and CVaR at level alpha (mc_risk). With
    opts.path_values the per-path P&L is returned as "pnl"."""
    mm = _Marshal(model, Payoff(MC_BASKET_CALL, 0.0), opts, n_paths)
    torch = _torch()
    if torch is not None:
        mm.co.hip_stream = torch.cuda.current_stream(ctx.device).cuda_stream
    m = _arr(strike_mult)
    q = _arr(quantity)
    if m.size != q.size or not 1 <= m.size <= MC_MAX_STRIKES:
        raise ValueError("strike_mult and quantity: 1..8 entries each, equal lengths")
    pf = _abi.McPortfolio()
    pf.n_strikes = m.size
    for i in range(m.size):
        pf.strike_mult[i] = m[i]
        pf.quantity[i] = q[i]
    if mu is not None:
        pf.mu = mm._ptr(_arr(mu), C.c_double)
    pf.alpha = alpha
    pnl = None
    if mm.opts.path_values:
        pnl = np.zeros(n_paths, np.float64)
        mm.co.path_values = mm._ptr(pnl, C.c_double)
    res = _abi.McRiskResult()
    st = _abi.load().mc_risk(ctx.handle, C.byref(mm.cm), C.byref(pf), n_paths, n_steps, seed,
                             C.byref(mm.co), C.byref(res))
    _check(ctx, st)
    out = {name: getattr(res, name) for name, _ in _abi.McRiskResult._fields_}
    if pnl is not None:
        out["pnl"] = pnl
    return out


def mc_price_qmc(ctx: Context, model: Model, payoff: Payoff, n_points: int, n_steps: int,
                 seed: int, n_replicates: int, opts: Options | None = None) -> dict:
    """Randomised Sobol' quasi-Monte Carlo basket price over n_replicates
    digital shifts (mc_price_qmc); with opts.path_values and one replicate
    the per-path channels come back as "path_values"."""
    mm = _Marshal(model, payoff, opts, n_points)
    torch = _torch()
    if torch is not None:
        mm.co.hip_stream = torch.cuda.current_stream(ctx.device).cuda_stream
    if mm.opts.path_values:
        mm.want_path_values(n_points, 3)
    res = _abi.McQmcResult()
    st = _abi.load().mc_price_qmc(ctx.handle, C.byref(mm.cm), C.byref(mm.cp), n_points, n_steps,
                                  seed, n_replicates, C.byref(mm.co), C.byref(res))
    _check(ctx, st)
    R = res.n_replicates
    out = {"price": res.price, "std_err": res.std_err, "geo_price": res.geo_price,
           "geo_std_err": res.geo_std_err, "n_replicates": R, "n_points": res.n_points,
           "replicate_price": list(res.replicate_price[:R]),
           "replicate_geo": list(res.replicate_geo[:R]), "kernel_ms": res.kernel_ms}
    if mm.path_buf is not None:
        out["path_values"] = mm.path_buf
    return out


@dataclass
class LsmSpec:
    """Bermudan contract and regression of mc_price_lsm."""
    payoff: int = MC_LSM_MAX_CALL
    K: float = 100.0
    dividend: float = 0.0
    n_dates: int = 9
    steps_per_date: int = 1
    degree: int = 2
    n_paths_oos: int = 0


def mc_price_lsm(ctx: Context, model: Model, spec: LsmSpec, n_paths: int, seed: int,
                 opts: Options | None = None, want_paths: bool = False) -> dict:
    """Longstaff-Schwartz price of a Bermudan option (mc_price_lsm): the
    in-sample and out-of-sample estimates, the regression coefficients of
    every date and, with want_paths, per-path cash flows and exercise dates."""
    payoff = Payoff(kind=MC_EURO_CALL, K=spec.K)
    mm = _Marshal(model, payoff, opts, n_paths)
    torch = _torch()
    if torch is not None:
        mm.co.hip_stream = torch.cuda.current_stream(ctx.device).cuda_stream
    cs = _abi.McLsmSpec(spec.payoff, spec.K, spec.dividend, spec.n_dates, spec.steps_per_date,
                        spec.degree, spec.n_paths_oos)
    res = _abi.McLsmResult()
    diag = None
    bufs = {}
    if want_paths:
        bufs = {"cash_flow": np.zeros(n_paths), "exercise_date": np.zeros(n_paths, np.int32),
                "oos_value": np.zeros(spec.n_paths_oos),
                "oos_exercise_date": np.zeros(spec.n_paths_oos, np.int32)}
        diag = _abi.McLsmPaths(
            bufs["cash_flow"].ctypes.data_as(C.POINTER(C.c_double)),
            bufs["exercise_date"].ctypes.data_as(C.POINTER(C.c_int32)),
            bufs["oos_value"].ctypes.data_as(C.POINTER(C.c_double)) if spec.n_paths_oos else None,
            bufs["oos_exercise_date"].ctypes.data_as(C.POINTER(C.c_int32))
            if spec.n_paths_oos else None)
    st = _abi.load().mc_price_lsm(ctx.handle, C.byref(mm.cm), C.byref(cs), n_paths, seed,
                                  C.byref(mm.co), C.byref(res),
                                  C.byref(diag) if diag is not None else None)
    _check(ctx, st)
    nf, M = res.n_features, spec.n_dates
    out = {"price": res.price, "std_err": res.std_err, "price_oos": res.price_oos,
           "std_err_oos": res.std_err_oos, "european": res.european,
           "european_se": res.european_se, "n_features": nf,
           "beta": np.array([[res.beta[j][k] for k in range(nf)] for j in range(M)]),
           "beta_valid": np.array(res.beta_valid[:M], np.int32),
           "n_itm": np.array(res.n_itm[:M], np.int64), "n_paths": res.n_paths,
           "n_paths_oos": res.n_paths_oos, "sim_ms": res.sim_ms, "regress_ms": res.regress_ms,
           "oos_ms": res.oos_ms, "update_ms": res.update_ms}
    out.update(bufs)
    return out


class PreparedPriceMulti:
    """mc_price_multi with its arguments marshalled once: calling it only
    invokes the C entry point, for tight repeated pricing loops."""

    def __init__(self, ctx: Context, model: Model, payoffs: Sequence[Payoff], n_paths: int,
                 n_steps: int, seed: int, opts: Options | None = None):
        self.ctx = ctx
        self.mm = _Marshal(model, list(payoffs), opts, n_paths)
        self.args = (n_paths, n_steps, seed)
        self.res = (_abi.McResult * len(payoffs))()
        self.fn = _abi.load().mc_price_multi
        self.cm = C.byref(self.mm.cm)
        self.co = C.byref(self.mm.co)
        self.n = len(payoffs)

    def __call__(self):
        st = self.fn(self.ctx.handle, self.cm, self.mm.cps, self.n, *self.args, self.co, self.res)
        _check(self.ctx, st)
        return self.res

    def results(self) -> list[dict]:
        return [_result(r) for r in self.res]


def mc_greeks_adjoint(ctx: Context, model: Model, payoff: Payoff, n_paths: int, n_steps: int,
                      seed: int, opts: Options | None = None, phase: int = MC_ADJ_FULL,
                      ckpt_every: int = 16, ckpt_ptr: int | None = None, ckpt_bytes: int = 0,
                      grad_out: float = 1.0) -> dict:
    mm = _Marshal(model, payoff, opts, n_paths)
    if mm.opts.path_values:
        nch = {MC_ADJ_FULL: 3, MC_ADJ_FWD: 1, MC_ADJ_REV: 2}[phase]
        mm.want_path_values(n_paths, nch)
    res = _abi.McResult()
    st = _abi.load().mc_greeks_adjoint(ctx.handle, C.byref(mm.cm), C.byref(mm.cp), n_paths,
                                       n_steps, seed, C.byref(mm.co), phase, ckpt_every,
                                       C.c_void_p(ckpt_ptr) if ckpt_ptr else None, ckpt_bytes,
                                       grad_out, C.byref(res))
    _check(ctx, st)
    out = _result(res)
    if mm.path_buf is not None:
        out["path_values"] = mm.path_buf
    return out


def mc_cv_train(ctx: Context, model: Model, payoff: Payoff, n_train: int, n_steps: int, seed: int,
                weights: np.ndarray, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, steps=2000,
                batch=1 << 16, hedge_every=1, prec=MC_FP32, decay_every=0, decay=1.0):
    mm = _Marshal(model, payoff, None, n_train)
    cfg = _abi.McAdamCfg(lr, beta1, beta2, eps, steps, batch, hedge_every, prec, decay_every,
                         decay)
    w = np.ascontiguousarray(weights, np.float32).copy()
    log = np.zeros(steps, np.float32)
    st = _abi.load().mc_cv_train(ctx.handle, C.byref(mm.cm), C.byref(mm.cp), n_train, n_steps,
                                 seed, C.byref(cfg), w.ctypes.data_as(_abi._fp),
                                 log.ctypes.data_as(_abi._fp))
    _check(ctx, st)
    return w, log


def mc_cv_loss_grad(ctx: Context, model: Model, payoff: Payoff, n_steps: int, seed: int, tag: int,
                    path0: int, batch: int, weights: np.ndarray, hedge_every=1, prec=MC_FP32):
    mm = _Marshal(model, payoff, None, batch)
    cfg = _abi.McAdamCfg(1e-3, 0.9, 0.999, 1e-8, 1, batch, hedge_every, prec)
    w = np.ascontiguousarray(weights, np.float32)
    loss = C.c_double()
    grad = np.zeros(MC_MLP_NPARAM, np.float32)
    st = _abi.load().mc_cv_loss_grad(ctx.handle, C.byref(mm.cm), C.byref(mm.cp), n_steps, seed,
                                     tag, path0, batch, C.byref(cfg), w.ctypes.data_as(_abi._fp),
                                     C.byref(loss), grad.ctypes.data_as(_abi._fp))
    _check(ctx, st)
    return loss.value, grad


def mc_philox_words(ctx: Context, seed: int, tag: int, paths, blocks) -> np.ndarray:
    paths = np.ascontiguousarray(paths, np.uint64)
    blocks = np.ascontiguousarray(blocks, np.uint64)
    out = np.zeros((paths.size, 4), np.uint32)
    st = _abi.load().mc_philox_words(ctx.handle, seed, tag, paths.size,
                                     paths.ctypes.data_as(_abi._u64p),
                                     blocks.ctypes.data_as(_abi._u64p),
                                     out.ctypes.data_as(_abi._u32p))
    _check(ctx, st)
    return out


def mc_normals(ctx: Context, seed: int, tag: int, path: int, k0: int, count: int,
               prec: int = MC_FP32) -> np.ndarray:
    out = np.zeros(count, np.float64)
    st = _abi.load().mc_normals(ctx.handle, seed, tag, path, k0, count, prec,
                                out.ctypes.data_as(_abi._dp))
    _check(ctx, st)
    return out


# ------------------------------------------------- autograd (adjoint) ----
def _make_pathwise_price():
    try:
        import torch
    except Exception:  # pragma: no cover
        return None

    class PathwisePrice(torch.autograd.Function):
        """Heston price as a differentiable function of (S0, v0).

        forward runs the adjoint kernel's forward sweep, which stores the
        checkpoints in a device buffer owned by this autograd node; backward
        runs the reverse sweep from those checkpoints and returns
        grad_out * (d price/d S0, d price/d v0).
        """

        @staticmethod
        def forward(actx, S0, v0, ctx: Context, model: Model, payoff: Payoff, n_paths: int,
                    n_steps: int, seed: int, opts: Options | None = None):
            m = Model(**{**model.__dict__, "S0": float(S0), "v0": float(v0)})
            nbytes = mc_adjoint_ckpt_bytes(n_paths, n_steps, 16)
            ck = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{ctx.device}")
            r = mc_greeks_adjoint(ctx, m, payoff, n_paths, n_steps, seed, opts, MC_ADJ_FWD, 16,
                                  ck.data_ptr(), nbytes)
            actx.saved = (ctx, m, payoff, n_paths, n_steps, seed, opts, ck, nbytes)
            return torch.tensor(r["price"], dtype=torch.float64)

        @staticmethod
        def backward(actx, grad_out):
            ctx, m, payoff, n_paths, n_steps, seed, opts, ck, nbytes = actx.saved
            r = mc_greeks_adjoint(ctx, m, payoff, n_paths, n_steps, seed, opts, MC_ADJ_REV, 16,
                                  ck.data_ptr(), nbytes, float(grad_out))
            g = torch.tensor
            return (g(r["delta"], dtype=torch.float64), g(r["vega"], dtype=torch.float64),
                    None, None, None, None, None, None, None)

    class TangentPrice(torch.autograd.Function):
        """Heston price as a differentiable function of (S0, v0), in forward
        mode.

        forward prices with the tangents of (ln S, v) with respect to S0 and
        v0 carried beside the state (mc_price, MC_GREEKS_TANGENT) and keeps
        the two derivatives; backward returns grad_out times them. One kernel
        and no checkpoint buffer; the derivatives are the adjoint's.
        """

        @staticmethod
        def forward(actx, S0, v0, ctx: Context, model: Model, payoff: Payoff, n_paths: int,
                    n_steps: int, seed: int, opts: Options | None = None):
            m = Model(**{**model.__dict__, "S0": float(S0), "v0": float(v0)})
            o = replace(opts if opts is not None else Options(),
                        greeks=MC_GREEK_DELTA | MC_GREEK_VEGA, greeks_method=MC_GREEKS_TANGENT)
            r = mc_price(ctx, m, payoff, n_paths, n_steps, seed, o)
            actx.saved = (r["delta"], r["vega"])
            return torch.tensor(r["price"], dtype=torch.float64)

        @staticmethod
        def backward(actx, grad_out):
            delta, dv0 = actx.saved
            g = float(grad_out)
            return (torch.tensor(g * delta, dtype=torch.float64),
                    torch.tensor(g * dv0, dtype=torch.float64),
                    None, None, None, None, None, None, None)

    return PathwisePrice, TangentPrice


PathwisePrice, TangentPrice = _make_pathwise_price() or (None, None)
