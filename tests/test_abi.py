"""Host-side checks of the C ABI: the library loads, exports every entry
point include/mcpath.h declares, and rejects bad arguments before touching a
device. No kernel runs here."""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

import paper_1906_02818_amd as mc
from paper_1906_02818_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1906_02818_amd import build as b
        b.build()


def test_library_exports_every_header_symbol():
    lib = _abi.load()
    names = _abi.header_symbols()
    assert "mc_price" in names and "mc_greeks_adjoint" in names and "mc_cv_train" in names
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)
    # ctypes signatures cover the header.
    assert set(names) == set(_abi.SIGNATURES), set(names) ^ set(_abi.SIGNATURES)


def test_struct_layout_matches_header(tmp_path):
    # Compile a tiny C program against the header and compare sizeof/offsetof.
    src = str(tmp_path / "abi_layout.c")
    with open(src, "w") as f:
        f.write('#include <stdio.h>\n#include <stddef.h>\n#include "mcpath.h"\n'
                'int main(){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(mc_model), '
                'sizeof(mc_payoff), sizeof(mc_options), sizeof(mc_result), sizeof(mc_adam_cfg),'
                ' offsetof(mc_options, path_values), offsetof(mc_result, cv_fallback));}\n')
    exe = src[:-2]
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    got = [int(x) for x in subprocess.run([exe], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(_abi.McModel), C.sizeof(_abi.McPayoff), C.sizeof(_abi.McOptions),
            C.sizeof(_abi.McResult), C.sizeof(_abi.McAdamCfg),
            _abi.McOptions.path_values.offset, _abi.McResult.cv_fallback.offset]
    assert got == want


def test_mlmc_struct_layout_matches_header(tmp_path):
    src = str(tmp_path / "abi_mlmc.c")
    with open(src, "w") as f:
        f.write('#include <stdio.h>\n#include <stddef.h>\n#include "mcpath.h"\n'
                'int main(){printf("%zu %zu %zu %zu %zu\\n", sizeof(mc_level), '
                'sizeof(mc_mlmc_result), offsetof(mc_mlmc_result, mean), '
                'offsetof(mc_mlmc_result, n_paths), offsetof(mc_mlmc_result, kernel_ms));}\n')
    exe = src[:-2]
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    got = [int(x) for x in subprocess.run([exe], capture_output=True, text=True,
                                          check=True).stdout.split()]
    R = _abi.McMlmcResult
    assert got == [C.sizeof(_abi.McLevel), C.sizeof(R), R.mean.offset, R.n_paths.offset,
                   R.kernel_ms.offset]


def test_risk_struct_layout_matches_header(tmp_path):
    src = str(tmp_path / "abi_risk.c")
    with open(src, "w") as f:
        f.write('#include <stdio.h>\n#include <stddef.h>\n#include "mcpath.h"\n'
                'int main(){printf("%zu %zu %zu %zu %zu\\n", sizeof(mc_portfolio), '
                'sizeof(mc_risk_result), offsetof(mc_portfolio, mu), '
                'offsetof(mc_portfolio, alpha), offsetof(mc_risk_result, select_ms));}\n')
    exe = src[:-2]
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    got = [int(x) for x in subprocess.run([exe], capture_output=True, text=True,
                                          check=True).stdout.split()]
    P, R = _abi.McPortfolio, _abi.McRiskResult
    assert got == [C.sizeof(P), C.sizeof(R), P.mu.offset, P.alpha.offset, R.select_ms.offset]


def test_qmc_struct_layout_matches_header(tmp_path):
    src = str(tmp_path / "abi_qmc.c")
    with open(src, "w") as f:
        f.write('#include <stdio.h>\n#include <stddef.h>\n#include "mcpath.h"\n'
                'int main(){printf("%zu %zu %zu\\n", sizeof(mc_qmc_result), '
                'offsetof(mc_qmc_result, replicate_geo), offsetof(mc_qmc_result, kernel_ms));}\n')
    exe = src[:-2]
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    got = [int(x) for x in subprocess.run([exe], capture_output=True, text=True,
                                          check=True).stdout.split()]
    R = _abi.McQmcResult
    assert got == [C.sizeof(R), R.replicate_geo.offset, R.kernel_ms.offset]


def test_lsm_struct_layout_matches_header(tmp_path):
    src = str(tmp_path / "abi_lsm.c")
    with open(src, "w") as f:
        f.write('#include <stdio.h>\n#include <stddef.h>\n#include "mcpath.h"\n'
                'int main(){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(mc_lsm_spec), '
                'offsetof(mc_lsm_spec, n_paths_oos), sizeof(mc_lsm_result), '
                'offsetof(mc_lsm_result, beta), offsetof(mc_lsm_result, n_itm), '
                'offsetof(mc_lsm_result, update_ms), sizeof(mc_lsm_paths), '
                'offsetof(mc_lsm_paths, oos_exercise_date));}\n')
    exe = src[:-2]
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    got = [int(x) for x in subprocess.run([exe], capture_output=True, text=True,
                                          check=True).stdout.split()]
    S, R, P = _abi.McLsmSpec, _abi.McLsmResult, _abi.McLsmPaths
    assert got == [C.sizeof(S), S.n_paths_oos.offset, C.sizeof(R), R.beta.offset,
                   R.n_itm.offset, R.update_ms.offset, C.sizeof(P), P.oos_exercise_date.offset]


def test_mlmc_allocation_is_the_lagrange_optimum():
    # N_l proportional to sqrt(V_l / C_l), scaled so that sum V_l / N_l hits
    # the target variance; checked against a direct minimisation.
    var = np.array([40.0, 0.5, 0.12, 0.03])
    cost = np.array([1.0, 3.0, 6.0, 12.0])
    eps = 0.01
    n = np.array(mc.mc_mlmc_allocate(var, cost, eps), np.float64)
    lam = np.sum(np.sqrt(var * cost)) / eps ** 2
    np.testing.assert_array_equal(n, np.ceil(lam * np.sqrt(var / cost)))
    assert np.sum(var / n) <= eps ** 2 * (1 + 1e-12)
    # Any other allocation with the same variance costs at least as much.
    rng = np.random.default_rng(0)
    for _ in range(200):
        x = n * np.exp(rng.normal(0, 0.3, n.size))
        x *= np.sum(var / x) / eps ** 2
        assert np.sum(x * cost) >= np.sum(n * cost) * (1 - 1e-6)
    assert mc.mc_mlmc_allocate([0.0, 1.0], [1.0, 1.0], 1.0) == [2, 2]


@pytest.mark.parametrize("var,cost,eps", [([1.0], [0.0], 0.1), ([-1.0], [1.0], 0.1),
                                          ([1.0], [1.0], 0.0), ([np.nan], [1.0], 0.1),
                                          ([1.0] * 9, [1.0] * 9, 0.1)])
def test_mlmc_allocation_rejects_bad_input(var, cost, eps):
    with pytest.raises(mc.McError) as e:
        mc.mc_mlmc_allocate(var, cost, eps)
    assert e.value.status == mc._abi.MC_ERR_INVALID_ARG


def test_binding_exports_every_name():
    missing = [n for n in mc.__all__ if not hasattr(mc, n)]
    assert not missing, missing


def test_status_strings():
    assert mc.mc_status_str(0) == "MC_OK"
    assert mc.mc_status_str(-2) == "MC_ERR_NOT_PD"
    assert mc.mc_status_str(-7) == "MC_ERR_WORKSPACE"


GBM = mc.Model(kind=mc.MC_GBM, S0=100.0, r=0.03, T=1.0, sigma=0.25)
HES = mc.Model(kind=mc.MC_HESTON, S0=100.0, r=0.02, T=1.0, v0=0.04, kappa=2.0, theta=0.04,
               xi=0.5, rho=-0.7)


@pytest.mark.parametrize("model,payoff,n_paths,n_steps,opts,want", [
    (GBM, mc.Payoff(mc.MC_EURO_CALL, 100.0), 1 << 10, 64, None, mc.MC_OK),
    (GBM, mc.Payoff(mc.MC_EURO_CALL, 100.0), 1, 64, None, mc._abi.MC_ERR_INVALID_ARG),
    (GBM, mc.Payoff(mc.MC_EURO_CALL, 100.0), 16, 0, None, mc._abi.MC_ERR_INVALID_ARG),
    (mc.Model(kind=mc.MC_GBM, S0=100.0, r=0.03, sigma=math.nan), mc.Payoff(), 16, 4, None,
     mc._abi.MC_ERR_INVALID_ARG),
    (mc.Model(kind=mc.MC_GBM, S0=-1.0, r=0.03, sigma=0.2), mc.Payoff(), 16, 4, None,
     mc._abi.MC_ERR_INVALID_ARG),
    (mc.Model(kind=mc.MC_GBM, S0=100.0, r=0.03, sigma=0.2, T=0.0), mc.Payoff(), 16, 4, None,
     mc._abi.MC_ERR_INVALID_ARG),
    (GBM, mc.Payoff(mc.MC_EURO_CALL, -5.0), 16, 4, None, mc._abi.MC_ERR_INVALID_ARG),
    (GBM, mc.Payoff(mc.MC_UO_BARRIER_CALL, 100.0, B=90.0), 16, 4, None,
     mc._abi.MC_ERR_INVALID_ARG),
    (GBM, mc.Payoff(mc.MC_UO_BARRIER_CALL, 100.0, B=130.0), 16, 4,
     mc.Options(greeks=mc.MC_GREEK_DELTA), mc._abi.MC_ERR_UNSUPPORTED),
    (GBM, mc.Payoff(mc.MC_EURO_CALL, 100.0, cv=mc.MC_CV_LEARNED), 16, 4, None,
     mc._abi.MC_ERR_UNSUPPORTED),
    (GBM, mc.Payoff(mc.MC_EURO_CALL, 100.0), 16, 4, mc.Options(prec=mc.MC_BF16_GEMM),
     mc._abi.MC_ERR_UNSUPPORTED),
    (GBM, mc.Payoff(mc.MC_EURO_CALL, 100.0), 16, 4, mc.Options(cv_hedge_every=0),
     mc._abi.MC_ERR_INVALID_ARG),
    (mc.Model(kind=mc.MC_GBM, S0=100.0, r=0.03, sigma=0.2, scheme=mc.MC_EULER_S),
     mc.Payoff(mc.MC_UO_BRIDGE_CALL, 100.0, B=130.0), 16, 4, None, mc._abi.MC_ERR_UNSUPPORTED),
    (HES, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0), 1 << 10, 256, None, mc.MC_OK),
    (mc.Model(kind=mc.MC_HESTON, S0=100.0, v0=-0.01, kappa=2, theta=0.04, xi=0.5, rho=-0.7),
     mc.Payoff(), 16, 4, None, mc._abi.MC_ERR_INVALID_ARG),
    (mc.Model(kind=mc.MC_HESTON, S0=100.0, v0=0.04, kappa=2, theta=0.04, xi=0.5, rho=1.0),
     mc.Payoff(), 16, 4, None, mc._abi.MC_ERR_INVALID_ARG),
    (HES, mc.Payoff(mc.MC_UO_BARRIER_CALL, 100.0, B=130.0), 16, 4, None,
     mc._abi.MC_ERR_UNSUPPORTED),
    (HES, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0), 16, 4,
     mc.Options(greeks=3, prec=mc.MC_FP64), mc._abi.MC_ERR_UNSUPPORTED),
    (HES, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0, cv=mc.MC_CV_LEARNED), 256, 16,
     mc.Options(cv_weights=np.zeros(mc.MC_MLP_NPARAM, np.float32),
                pilot_paths=mc.MC_PILOT_IN_SAMPLE), mc._abi.MC_ERR_UNSUPPORTED),
    (HES, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0, cv=mc.MC_CV_LEARNED), 256, 16,
     mc.Options(cv_weights=np.zeros(mc.MC_MLP_NPARAM, np.float32), cv_beta=1.0,
                pilot_paths=mc.MC_PILOT_IN_SAMPLE), mc.MC_OK),
])
def test_validation_without_device(model, payoff, n_paths, n_steps, opts, want):
    assert mc.mc_validate(model, payoff, n_paths, n_steps, opts) == want


def test_create_without_device_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(mc.McError) as e:
        mc.mc_create(0)
    assert e.value.status == mc._abi.MC_ERR_NO_DEVICE


def test_channel_names_and_sizes():
    names = mc.mc_path_channels(GBM, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0,
                                               cv=mc.MC_CV_GEO_ASIAN))
    assert names == ["asian", "geo", "uo"]
    names = mc.mc_path_channels(GBM, mc.Payoff(mc.MC_EURO_CALL, 100.0),
                                mc.Options(prec=mc.MC_FP64, greeks=3))
    assert names == ["euro", "euro_delta", "euro_vega"]
    names = mc.mc_path_channels(GBM, mc.Payoff(mc.MC_UO_BRIDGE_CALL, 100.0, B=130.0))
    assert names[4] == "uo_bridge" and len(names) == 9
    assert mc.mc_path_channels(HES, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0),
                               mc.Options(greeks=3)) == ["asian", "asian_delta", "asian_dv0"]
    # Checkpoints: one per `every` steps, (2 per checkpoint + 1) FP32 rows per
    # path; the period is even, 2..16.
    assert mc.mc_adjoint_ckpt_bytes(1000, 256, 16) == (2 * 16 + 1) * 1000 * 4
    assert mc.mc_adjoint_ckpt_bytes(1000, 250, 16) == (2 * 16 + 1) * 1000 * 4
    assert mc.mc_adjoint_ckpt_bytes(1000, 256, 8) == (2 * 32 + 1) * 1000 * 4
    assert mc.mc_adjoint_ckpt_bytes(1000, 7, 2) == (2 * 4 + 1) * 1000 * 4
    for bad in (0, 1, 3, 18, 32):
        assert mc.mc_adjoint_ckpt_bytes(1000, 256, bad) == 0
    # The one-launch adjoint keeps up to 16 checkpoints in LDS: no workspace
    # for them at 256 steps; above that the buffer is part of the workspace.
    hp = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0)
    assert mc.mc_workspace_bytes(HES, hp, 1 << 20, 256, mc.Options(greeks=3)) < (1 << 20)
    assert mc.mc_workspace_bytes(HES, hp, 1 << 20, 512, mc.Options(greeks=3)) > \
        mc.mc_adjoint_ckpt_bytes(1 << 20, 512, 16)
    ws = mc.mc_workspace_bytes(GBM, mc.Payoff(mc.MC_EURO_CALL, 100.0), 1 << 20, 64)
    assert ws >= (1 << 20) // 256 * 4 * 8     # 4 moments per block for one channel


def _basket(d=32, corr=None, **kw):
    import synth
    sigma, c, _ = synth.basket_market(d)
    return mc.Model(kind=mc.MC_GBM_BASKET, S0=np.full(d, 100.0), r=0.05, T=1.0, sigma=sigma,
                    corr=c if corr is None else corr, **kw)


def test_basket_validation_without_device():
    f = mc.Payoff(mc.MC_BASKET_CALL, 100.0)
    assert mc.mc_validate(_basket(), f, 1024, 100, mc.Options(prec=mc.MC_BF16_GEMM)) == mc.MC_OK
    assert mc.mc_validate(_basket(256), f, 1024, 100, mc.Options(prec=mc.MC_FP16_GEMM)) == mc.MC_OK
    # Not positive definite: an off-diagonal above 1.
    m = _basket()
    bad = np.array(m.corr)
    bad[0, 1] = bad[1, 0] = 1.2
    assert mc.mc_validate(_basket(corr=bad), f, 1024, 10) == mc._abi.MC_ERR_NOT_PD
    # Singular (two identical assets) is not positive definite either.
    sing = np.array(m.corr)
    sing[1, :] = sing[0, :]
    sing[:, 1] = sing[:, 0]
    sing[1, 1] = 1.0
    assert mc.mc_validate(_basket(corr=sing), f, 1024, 10) == mc._abi.MC_ERR_NOT_PD
    asym = np.array(m.corr)
    asym[0, 1] += 1e-3
    assert mc.mc_validate(_basket(corr=asym), f, 1024, 10) == mc._abi.MC_ERR_INVALID_ARG
    d20 = mc.Model(kind=mc.MC_GBM_BASKET, S0=np.full(20, 100.0), sigma=np.full(20, 0.2),
                   corr=np.eye(20))
    assert mc.mc_validate(d20, f, 1024, 10) == mc._abi.MC_ERR_UNSUPPORTED
    assert mc.mc_validate(_basket(), f, 1024, 10, mc.Options(prec=mc.MC_FP64)) == \
        mc._abi.MC_ERR_UNSUPPORTED
    assert mc.mc_validate(_basket(), f, 1024, 10, mc.Options(greeks=mc.MC_GREEK_VEGA)) == \
        mc._abi.MC_ERR_UNSUPPORTED
    assert mc.mc_validate(_basket(), mc.Payoff(mc.MC_EURO_CALL, 100.0), 1024, 10) == \
        mc._abi.MC_ERR_UNSUPPORTED
    assert mc.mc_path_channels(_basket(), f) == ["basket", "geo_basket", "basket_delta0"]


def test_learned_cv_validation_without_device():
    w = np.zeros(4545, np.float32)
    f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, 100.0, cv=mc.MC_CV_LEARNED)
    assert mc.mc_validate(HES, f, 1024, 256, mc.Options(cv_weights=w)) == mc.MC_OK
    assert mc.mc_validate(HES, f, 1024, 256, mc.Options(cv_weights=w, prec=mc.MC_BF16_GEMM)) \
        == mc.MC_OK
    assert mc.mc_validate(HES, f, 1024, 256) == mc._abi.MC_ERR_INVALID_ARG          # no weights
    assert mc.mc_validate(HES, f, 1024, 256, mc.Options(cv_weights=w, prec=mc.MC_FP64)) == \
        mc._abi.MC_ERR_UNSUPPORTED
    assert mc.mc_validate(HES, mc.Payoff(mc.MC_EURO_CALL, 100.0, cv=mc.MC_CV_LEARNED), 1024, 256,
                          mc.Options(cv_weights=w)) == mc._abi.MC_ERR_UNSUPPORTED
    assert mc.mc_validate(HES, f, 1024, 256, mc.Options(cv_weights=w, greeks=1)) == \
        mc._abi.MC_ERR_UNSUPPORTED
    h0 = mc.Model(kind=mc.MC_HESTON, S0=100.0, v0=0.04, kappa=2, theta=0.0, xi=0.5, rho=-0.7)
    assert mc.mc_validate(h0, f, 1024, 256, mc.Options(cv_weights=w)) == mc._abi.MC_ERR_INVALID_ARG
    assert mc.mc_path_channels(HES, f, mc.Options(cv_weights=w)) == \
        ["asian", "hedge_pnl", "asian_minus_hedge"]
