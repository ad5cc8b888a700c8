"""ctypes mirror of include/mcpath.h. Marshalling only: no arithmetic of the
method lives here."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcpath.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mcpath.h")

# enums
MC_OK, MC_ERR_INVALID_ARG, MC_ERR_NOT_PD, MC_ERR_NO_DEVICE = 0, -1, -2, -3
MC_ERR_OOM, MC_ERR_DEVICE, MC_ERR_UNSUPPORTED, MC_ERR_WORKSPACE = -4, -5, -6, -7
MC_GBM, MC_GBM_BASKET, MC_HESTON = 1, 2, 3
MC_LOG_EULER, MC_EULER_S = 0, 1
MC_FP64, MC_FP32, MC_BF16_GEMM, MC_FP16_GEMM, MC_BF16X2_GEMM = 0, 1, 2, 3, 4
MC_EURO_CALL, MC_ASIAN_ARITH_CALL, MC_ASIAN_GEO_CALL = 1, 2, 3
MC_UO_BARRIER_CALL, MC_BASKET_CALL, MC_UO_BRIDGE_CALL = 4, 5, 6
MC_CV_NONE, MC_CV_GEO_ASIAN, MC_CV_LEARNED = 0, 1, 2
MC_GREEK_DELTA, MC_GREEK_VEGA = 1, 2
MC_ADJ_FULL, MC_ADJ_FWD, MC_ADJ_REV = 0, 1, 2
MC_GREEKS_PATHWISE, MC_GREEKS_FD_CRN, MC_GREEKS_TANGENT = 0, 1, 2
MC_MLP_NPARAM = 4545
MC_PILOT_IN_SAMPLE = (1 << 64) - 1
MC_MLMC_MAX_LEVELS = 8
MC_MAX_STRIKES = 8
MC_QMC_MAX_REPLICATES = 64
MC_COUPLE_NONE, MC_COUPLE_PRECISION, MC_COUPLE_TIME = 0, 1, 2
MC_LSM_MAX_DATES = 64
MC_LSM_MAX_FEATURES = 11
MC_LSM_MAX_CALL, MC_LSM_BASKET_PUT, MC_LSM_BASKET_CALL = 1, 2, 3

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_u64p = C.POINTER(C.c_uint64)
_u32p = C.POINTER(C.c_uint32)


class McModel(C.Structure):
    _fields_ = [("kind", C.c_int), ("dim", C.c_uint32), ("r", C.c_double), ("T", C.c_double),
                ("S0", _dp), ("sigma", _dp), ("corr", _dp), ("v0", C.c_double),
                ("kappa", C.c_double), ("theta", C.c_double), ("xi", C.c_double),
                ("rho", C.c_double), ("scheme", C.c_int)]


class McPayoff(C.Structure):
    _fields_ = [("kind", C.c_int), ("K", C.c_double), ("B", C.c_double), ("weights", _dp),
                ("cv", C.c_int)]


class McOptions(C.Structure):
    _fields_ = [("prec", C.c_int), ("greeks", C.c_uint32), ("path_offset", C.c_uint64),
                ("stream_tag", C.c_uint32), ("hip_stream", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("cv_weights", _fp), ("cv_hedge_every", C.c_uint32), ("cv_beta", C.c_double),
                ("pilot_paths", C.c_uint64), ("path_values", _dp),
                ("greeks_method", C.c_uint32), ("fd_rel_step", C.c_double)]


class McResult(C.Structure):
    _fields_ = [("price", C.c_double), ("std_err", C.c_double), ("variance", C.c_double),
                ("delta", C.c_double), ("delta_se", C.c_double), ("vega", C.c_double),
                ("vega_se", C.c_double), ("plain_price", C.c_double),
                ("plain_std_err", C.c_double), ("cv_beta", C.c_double), ("vrf", C.c_double),
                ("n_paths", C.c_uint64), ("n_nonfinite", C.c_uint64),
                ("kernel_ms", C.c_double), ("cv_fallback", C.c_int), ("greeks_method", C.c_int)]


class McLevel(C.Structure):
    _fields_ = [("n_steps", C.c_uint32), ("prec", C.c_int), ("n_paths", C.c_uint64)]


_L = MC_MLMC_MAX_LEVELS


class McMlmcResult(C.Structure):
    _fields_ = [("price", C.c_double), ("std_err", C.c_double), ("n_levels", C.c_uint32),
                ("coupling", C.c_int * _L), ("mean", C.c_double * _L),
                ("variance", C.c_double * _L), ("fine_mean", C.c_double * _L),
                ("coarse_mean", C.c_double * _L), ("n_paths", C.c_uint64 * _L),
                ("kernel_ms", C.c_double * _L)]


class McPortfolio(C.Structure):
    _fields_ = [("n_strikes", C.c_uint32), ("strike_mult", C.c_double * MC_MAX_STRIKES),
                ("quantity", C.c_double * MC_MAX_STRIKES), ("mu", _dp), ("alpha", C.c_double)]


class McRiskResult(C.Structure):
    _fields_ = [("var", C.c_double), ("cvar", C.c_double), ("quantile_pnl", C.c_double),
                ("pnl_mean", C.c_double), ("pnl_std_err", C.c_double), ("premium", C.c_double),
                ("k", C.c_uint64), ("n_tail", C.c_uint64), ("n_paths", C.c_uint64),
                ("kernel_ms", C.c_double), ("select_ms", C.c_double)]


class McQmcResult(C.Structure):
    _fields_ = [("price", C.c_double), ("std_err", C.c_double), ("geo_price", C.c_double),
                ("geo_std_err", C.c_double), ("n_replicates", C.c_uint32),
                ("n_points", C.c_uint64),
                ("replicate_price", C.c_double * MC_QMC_MAX_REPLICATES),
                ("replicate_geo", C.c_double * MC_QMC_MAX_REPLICATES),
                ("kernel_ms", C.c_double)]


class McLsmSpec(C.Structure):
    _fields_ = [("payoff", C.c_int), ("K", C.c_double), ("dividend", C.c_double),
                ("n_dates", C.c_uint32), ("steps_per_date", C.c_uint32), ("degree", C.c_uint32),
                ("n_paths_oos", C.c_uint64)]


class McLsmResult(C.Structure):
    _fields_ = [("price", C.c_double), ("std_err", C.c_double), ("price_oos", C.c_double),
                ("std_err_oos", C.c_double), ("european", C.c_double),
                ("european_se", C.c_double), ("n_features", C.c_uint32),
                ("beta", (C.c_double * MC_LSM_MAX_FEATURES) * MC_LSM_MAX_DATES),
                ("beta_valid", C.c_int * MC_LSM_MAX_DATES),
                ("n_itm", C.c_uint64 * MC_LSM_MAX_DATES),
                ("n_paths", C.c_uint64), ("n_paths_oos", C.c_uint64), ("sim_ms", C.c_double),
                ("regress_ms", C.c_double), ("oos_ms", C.c_double), ("update_ms", C.c_double)]


class McLsmPaths(C.Structure):
    _fields_ = [("cash_flow", C.POINTER(C.c_double)), ("exercise_date", C.POINTER(C.c_int32)),
                ("oos_value", C.POINTER(C.c_double)),
                ("oos_exercise_date", C.POINTER(C.c_int32))]


class McAdamCfg(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("steps", C.c_uint32), ("batch", C.c_uint64),
                ("hedge_every", C.c_uint32), ("prec", C.c_int), ("decay_every", C.c_uint32),
                ("decay", C.c_double)]


_P = C.POINTER
SIGNATURES = {
    "mc_create": (C.c_int, [_P(C.c_void_p), C.c_int]),
    "mc_destroy": (C.c_int, [C.c_void_p]),
    "mc_options_default": (None, [_P(McOptions)]),
    "mc_validate": (C.c_int, [C.c_void_p, _P(McModel), _P(McPayoff), C.c_uint64, C.c_uint32,
                              _P(McOptions)]),
    "mc_workspace_bytes": (C.c_size_t, [_P(McModel), _P(McPayoff), C.c_uint64, C.c_uint32,
                                        _P(McOptions)]),
    "mc_price": (C.c_int, [C.c_void_p, _P(McModel), _P(McPayoff), C.c_uint64, C.c_uint32,
                           C.c_uint64, _P(McOptions), _P(McResult)]),
    "mc_noalloc_scratch_bytes": (C.c_size_t, []),
    "mc_price_noalloc": (C.c_int, [C.c_void_p, _P(McModel), _P(McPayoff), C.c_uint64, C.c_uint32,
                                   C.c_uint64, _P(McOptions), _P(McResult)]),
    "mc_price_multi": (C.c_int, [C.c_void_p, _P(McModel), _P(McPayoff), C.c_uint32, C.c_uint64,
                                 C.c_uint32, C.c_uint64, _P(McOptions), _P(McResult)]),
    "mc_path_channels": (C.c_uint32, [_P(McModel), _P(McPayoff), _P(McOptions)]),
    "mc_path_channel_name": (C.c_char_p, [_P(McModel), _P(McPayoff), _P(McOptions), C.c_uint32]),
    "mc_adjoint_ckpt_bytes": (C.c_size_t, [C.c_uint64, C.c_uint32, C.c_uint32]),
    "mc_greeks_adjoint": (C.c_int, [C.c_void_p, _P(McModel), _P(McPayoff), C.c_uint64, C.c_uint32,
                                    C.c_uint64, _P(McOptions), C.c_int, C.c_uint32, C.c_void_p,
                                    C.c_size_t, C.c_double, _P(McResult)]),
    "mc_cv_train": (C.c_int, [C.c_void_p, _P(McModel), _P(McPayoff), C.c_uint64, C.c_uint32,
                              C.c_uint64, _P(McAdamCfg), _fp, _fp]),
    "mc_cv_loss_grad": (C.c_int, [C.c_void_p, _P(McModel), _P(McPayoff), C.c_uint32, C.c_uint64,
                                  C.c_uint32, C.c_uint64, C.c_uint64, _P(McAdamCfg), _fp, _dp,
                                  _fp]),
    "mc_philox_words": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint64, _u64p, _u64p,
                                  _u32p]),
    "mc_normals": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64,
                             C.c_uint64, C.c_int, _dp]),
    "mc_price_mlmc": (C.c_int, [C.c_void_p, _P(McModel), _P(McPayoff), C.c_uint32, _P(McLevel),
                                C.c_uint64, _P(McOptions), _P(McMlmcResult)]),
    "mc_mlmc_allocate": (C.c_int, [C.c_uint32, _dp, _dp, C.c_double, _u64p]),
    "mc_risk": (C.c_int, [C.c_void_p, _P(McModel), _P(McPortfolio), C.c_uint64, C.c_uint32,
                          C.c_uint64, _P(McOptions), _P(McRiskResult)]),
    "mc_price_qmc": (C.c_int, [C.c_void_p, _P(McModel), _P(McPayoff), C.c_uint64, C.c_uint32,
                               C.c_uint64, C.c_uint32, _P(McOptions), _P(McQmcResult)]),
    "mc_price_lsm": (C.c_int, [C.c_void_p, _P(McModel), _P(McLsmSpec), C.c_uint64, C.c_uint64,
                               _P(McOptions), _P(McLsmResult), _P(McLsmPaths)]),
    "mc_status_str": (C.c_char_p, [C.c_int]),
    "mc_last_error": (C.c_char_p, [C.c_void_p]),
}

_lib = None


def load():
    """Loads libmcpath.so; raises when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def header_symbols() -> list[str]:
    """Function names declared in include/mcpath.h."""
    import re
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mc_[a-z0-9_]+)\s*\(", text)))
