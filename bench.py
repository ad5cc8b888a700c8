"""Benchmark of the Monte Carlo path engine on one MI355X.

Default workload (the metric's configuration): arithmetic-average Asian call
(with the geometric-Asian control variate) and discretely monitored
up-and-out call (B = 130) priced on the same 1-D GBM paths: S0 = K = 100,
r = 0.03, sigma = 0.25, T = 1, 252 log-Euler steps, 2^24 paths, FP32 path
state, FP64 cross-path reduction, Philox4x32-10 seed 1234. One step of the
benchmark is one full pricing pass: the path kernel (random numbers,
Euler-Maruyama steps, path functionals, payoffs, block moments), the
fixed-order final reduction and the read-back of the moments. Inputs are
parameters only, so nothing is staged from the host in the timed region.

Prints one JSON line. `roofline` reports the dominant kernel against the
ALU issue peak (the path kernels read and write no HBM per step);
`time_to_1bp` compares, after the timed region, plain FP32 Monte Carlo with
the learned control variate (BF16 matrix products) on the Heston Asian
call; `cpu_baseline` times the FP64 oracle on a bounded sample of the same
workload on the host cores.

Other configurations, for profiling (--workload): european (FP64 with
pathwise greeks), basket (d = 256, --prec), heston_adjoint, learned_cv.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz; the FP32 vector peak (157.3 TFLOP/s) is 128
# FMA lanes per clock per CU, the unit ("slot") of the ALU roofline.
N_CU, CLOCK_HZ, FMA_LANES_PER_CLK = 256, 2.4e9, 128
ALU_PEAK_SLOTS = N_CU * CLOCK_HZ * FMA_LANES_PER_CLK      # 7.86e13 slots/s
MFMA_PEAK = {"fp32": 157.3e12, "bf16": 2.5e15, "fp16": 2.5e15, "bf16x2": 2.5e15}
HBM_PEAK = 8.0e12                                           # bytes/s
# One v_mfma_f32_32x32x16 (BF16/FP16) occupies a SIMD for about 35.5 cycles
# (isa_rates.hip, matrix core alone; nominal 8 passes = 32), and on one SIMD
# the matrix core overlaps vector issue by only ~12 % (same probe), so the
# bound of a kernel issuing both is VALU issue time + MFMA time.
MFMA_CYCLES_32X32X16 = 35.5
N_SIMD = 4 * N_CU


def _mfma_share(n_mfma, kernel_ms):
    """Fraction of the kernel time the SIMDs spend in n_mfma 32x32x16 MFMAs."""
    return n_mfma * MFMA_CYCLES_32X32X16 / N_SIMD / CLOCK_HZ / (kernel_ms * 1e-3)

# Issue cost of each instruction class on gfx950 in "slots": wave64 FMA
# issues at the FP32 vector peak (2 per clock per CU). Costs are 2 divided
# by the wave64 issue rate per clock per CU that
# paper_1906_02818_amd/isa_rates.hip measures in isolation
# (profiles/isa_rates.txt). An FP32 FMA issues at 1.77 per clock, so it
# costs 1.13; other single-pass 32-bit operations (xor, shift, compare,
# alignbit) are charged the same. The isolated three-input xor measures half
# that rate (2.08), but in the Philox rounds it replaced two xors and made
# the kernels faster, so it is charged as one single-pass operation, the
# lower (conservative) figure.
COST_FP32 = 1.13     # add, mul, fma
COST_INT = 1.13      # xor, shift, compare, alignbit
COST_BITOP3 = 1.13   # v_bitop3_b32 (three-input xor)
COST_MUL64 = 3.01    # 32x32->64-bit product (v_mad_u64_u32): 4.14 with its xor, minus 1.13
COST_TRANS = 4.09    # v_exp / sin / cos / sqrt / rcp _f32
COST_LOG = 4.09      # v_log_f32: between 4.09 and 6.06 - 1.13; the lower figure
COST_FP64 = 2.40     # v_fma_f64


def slots(mul64=0.0, trans=0.0, log=0.0, intops=0.0, fp32=0.0, fp64=0.0, bitop3=0.0):
    return (mul64 * COST_MUL64 + trans * COST_TRANS + log * COST_LOG + intops * COST_INT
            + fp32 * COST_FP32 + fp64 * COST_FP64 + bitop3 * COST_BITOP3)


# One FP32 normal: a quarter of a Philox4x32-10 block (10 rounds of 2 mul64
# and 2 three-input xors), the uniform (one alignbit, one sub) and half of a
# Box-Muller pair (log, sqrt, sin, cos and 3 mul). Where every lane of a wave
# draws the same block index at a step (one path per lane), round 1's two
# products (block index; the path's high word, the same for every path below
# 2^32) and round 2's second (fed only by round 1's uniform results) do not
# depend on the path: 17 of the 20 products are per-path work, the count the
# compiled kernels issue. The basket's lanes draw two block indices per step,
# so all 20 are.
NORMAL = dict(mul64=17 / 4, log=0.5, trans=1.5, bitop3=5.0, intops=1.0, fp32=1.0 + 1.5)
NORMAL_BASKET = dict(NORMAL, mul64=20 / 4)


def _add(*ds):
    out = {}
    for d in ds:
        for k, v in d.items():
            out[k] = out.get(k, 0.0) + v
    return out


# Algorithmic work per path-step (asset-path-step for the basket).
SLOTS_ASIAN_BARRIER = slots(**_add(NORMAL, dict(trans=1.0, intops=1.0, fp32=4.0)))
#   normal; step fma + add; Asian exp2 + add; geometric add; barrier compare
SLOTS_HESTON = slots(**_add(NORMAL, NORMAL, dict(trans=2.0, fp32=11.0)))
#   2 normals; v+ max, sqrt(v+ dt), Zs (mul, fma), ln S (fma, add, fma),
#   v (fma, fma, mul), Asian exp2 + add
SLOTS_HESTON_REVERSE = slots(trans=2.0, fp32=6.0, fp64=3.0)
#   per step of the reverse sweep: sqrt, rcp, 6 FP32 ops, 3 FP64 ops
SLOTS_ASSET_STEP = slots(**_add(NORMAL_BASKET, dict(intops=0.5)))
#   per asset-path-step of the basket: one normal and half a 16-bit pack
SLOTS_TANH = slots(trans=2.0, fp32=3.0)
#   tanh(x + b): fma, exp2, add, rcp, fma
SLOTS_SIGM = slots(trans=2.0, fp32=2.0)
#   (1 + tanh(x + b)) / 2, the form layer 3 takes where only Delta is needed


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(c, budget_s=12.0):
    """FP64 oracle on the host cores over a bounded sample of the workload."""
    import oracle
    n = c["n_steps"]
    t0 = time.perf_counter()
    probe = 1 << 12

    def run(k):
        # The payoff channels the timed step computes (arithmetic and
        # geometric Asian, discrete up-and-out barrier; the European payoff
        # and S_T come with them): no tangents, bridge stream or margins.
        oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], c["B"], n, k, 1234,
                   payoffs_only=True)
    run(probe)
    dt = time.perf_counter() - t0
    n_paths = int(max(probe, min(c["n_paths"], probe * budget_s / max(dt, 1e-6))))
    n_paths = 1 << int(math.log2(n_paths))
    t0 = time.perf_counter()
    run(n_paths)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_paths * n / dt, "unit": "path-steps/s", "cores": threads,
            "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"{n_paths} of {c['n_paths']} paths x {n} steps of the GBM oracle (FP64), "
                      f"channels arithmetic Asian, geometric Asian, discrete up-and-out barrier "
                      f"(with the European payoff and S_T they share), {dt:.1f} s"}


def _oracle_sample(fn, probe, n_max, budget_s=8.0):
    """Runs fn(n) on a probe of n units, then once more on a power-of-two
    count sized to about budget_s seconds (at most n_max); returns (n, s)."""
    t0 = time.perf_counter()
    fn(probe)
    dt = time.perf_counter() - t0
    n = int(max(probe, min(n_max, probe * budget_s / max(dt, 1e-6))))
    n = 1 << int(math.log2(n))
    t0 = time.perf_counter()
    fn(n)
    return n, time.perf_counter() - t0


def _cpu_entry(value, unit, sample, **extra):
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict({"value": value, "unit": unit, "cores": threads, "kind": "oracle",
                 "cpu_model": _cpu_model(), "sample": sample}, **extra)


def _basket_oracle_inputs(synth, d):
    import numpy as np
    import oracle
    sigma, corr, _ = synth.basket_market(d)
    return sigma, oracle.cholesky(corr), np.full(d, 1.0 / d)


def _paths_for(se_target, sigma):
    n = int(math.ceil((sigma / se_target) ** 2))
    return max(256, (n + 255) // 256 * 256)


def _heston_model(mc, synth):
    H = synth.HESTON
    return mc.Model(kind=mc.MC_HESTON, S0=H["S0"], r=H["r"], T=H["T"], v0=H["v0"],
                    kappa=H["kappa"], theta=H["theta"], xi=H["xi"], rho=H["rho"])


def _timed(torch, fn):
    """One timed call, with Python's garbage collector paused (see _repeat)."""
    import gc
    gc_was_on = gc.isenabled()
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0
    finally:
        if gc_was_on:
            gc.enable()


def _pilot_then_run(torch, pilot_fn, run_fn, reps=3):
    """Time to 1 bp of one estimator: a pilot sizes N*, a run of N* paths
    follows; both are timed. One untimed pair first (the workspace grows to
    the run's size once, as in any later pricing), then `reps` timed pairs;
    returns the pair with the median total and every total."""
    def pair():
        pil, t_pil = _timed(torch, pilot_fn)
        N = _paths_for(1e-4 * pil["price"], math.sqrt(pil["variance"]))
        run, t_run = _timed(torch, lambda: run_fn(N))
        return pil, t_pil, N, run, t_run
    pair()
    pairs = sorted((pair() for _ in range(reps)), key=lambda x: x[1] + x[4])
    pil, t_pil, N, run, t_run = pairs[len(pairs) // 2]
    return pil, t_pil, N, run, t_run, [x[1] + x[4] for x in pairs]


def time_to_1bp(ctx, mc, synth, torch, hedge_every=16, adam_steps=None):
    """Time to a Heston-Asian price whose standard error is 1 bp of the price
    (1e-4 x price), plain FP32 Monte Carlo against the learned control
    variate with BF16 matrix products. Each estimator: a 2^20-path pilot on
    stream tag 1 sizes N* = (s / (1e-4 p))^2, then one run of N* paths on
    tag 0; both are timed (median of three pairs after an untimed one, see
    _pilot_then_run). The hedge network is trained beforehand (the Adam
    recipe of synth.LEARNED_CV: 2000 steps with a stepped learning rate,
    minibatch 2^15 from a fixed 2^20-path set on tag 2); its training time
    is reported separately and added in `total_incl_train_s`.
    """
    import numpy as np
    H = synth.HESTON
    cv = synth.LEARNED_CV
    if adam_steps is None:
        adam_steps = cv["adam_steps"]
    n = H["n_steps"]
    model = _heston_model(mc, synth)
    plain_f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, H["K"])
    cv_f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, H["K"], cv=mc.MC_CV_LEARNED)
    out = {"workload": f"Heston arithmetic-Asian call, {n} steps; target SE = 1e-4 x price",
           "hedge_every": hedge_every}
    pil, t_pil, N_plain, run, t_run, totals = _pilot_then_run(
        torch, lambda: mc.mc_price(ctx, model, plain_f, 1 << 20, n, synth.SEED,
                                   mc.Options(stream_tag=1)),
        lambda N: mc.mc_price(ctx, model, plain_f, N, n, synth.SEED))
    out["plain_fp32"] = {"pilot_s": t_pil, "n_paths": N_plain, "run_s": t_run,
                         "total_s": t_pil + t_run, "totals_s": totals, "price": run["price"],
                         "std_err": run["std_err"], "kernel_ms": run["kernel_ms"]}
    th0 = synth.glorot_mlp()
    (w, log), t_train = _timed(torch, lambda: mc.mc_cv_train(
        ctx, model, cv_f, cv["n_train"], n, synth.SEED, th0, lr=cv["lr"], beta2=cv["beta2"],
        steps=adam_steps, batch=cv["batch"], hedge_every=hedge_every, prec=mc.MC_BF16_GEMM,
        decay_every=cv["decay_every"], decay=cv["decay"]))

    def opts(tag):
        return mc.Options(prec=mc.MC_BF16_GEMM, cv_weights=w, cv_hedge_every=hedge_every,
                          cv_beta=1.0, stream_tag=tag)

    pil, t_pil, N_cv, run, t_run, totals_cv = _pilot_then_run(
        torch, lambda: mc.mc_price(ctx, model, cv_f, 1 << 20, n, synth.SEED, opts(1)),
        lambda N: mc.mc_price(ctx, model, cv_f, N, n, synth.SEED, opts(0)))
    out["learned_cv_bf16"] = {"train_s": t_train, "adam_steps": adam_steps,
                              "adam": {"lr": cv["lr"], "beta2": cv["beta2"], "batch": cv["batch"],
                                       "decay": cv["decay"], "decay_every": cv["decay_every"]},
                              "loss_first": float(log[0]), "loss_last": float(np.mean(log[-20:])),
                              "pilot_s": t_pil, "pilot_vrf": pil["vrf"], "n_paths": N_cv,
                              "run_s": t_run, "total_s": t_pil + t_run, "totals_s": totals_cv,
                              "total_incl_train_s": t_train + t_pil + t_run,
                              "price": run["price"], "std_err": run["std_err"],
                              "vrf": run["vrf"], "plain_price_same_paths": run["plain_price"],
                              "kernel_ms": run["kernel_ms"]}
    # The trained network evaluated once on 2^24 fresh paths (stream tag 8,
    # used by nothing else): its variance-reduction factor against plain
    # Monte Carlo on the same paths.
    ev, t_ev = _timed(torch, lambda: mc.mc_price(ctx, model, cv_f, 1 << 24, n, synth.SEED,
                                                 opts(8)))
    out["learned_cv_bf16"]["fresh_2p24"] = {
        "stream_tag": 8, "n_paths": 1 << 24, "price": ev["price"], "std_err": ev["std_err"],
        "vrf": ev["vrf"], "plain_price": ev["plain_price"], "plain_std_err": ev["plain_std_err"],
        "run_s": t_ev, "kernel_ms": ev["kernel_ms"]}
    out["speedup_excl_train"] = out["plain_fp32"]["total_s"] / out["learned_cv_bf16"]["total_s"]
    out["speedup_incl_train"] = (out["plain_fp32"]["total_s"]
                                 / out["learned_cv_bf16"]["total_incl_train_s"])
    # Both estimators' path counts scale as 1 / SE^2 while the training cost
    # is fixed: the learned CV, training included, is faster for standard
    # errors below this many basis points of the price.
    gain = out["plain_fp32"]["total_s"] - out["learned_cv_bf16"]["total_s"]
    out["break_even_se_bp"] = math.sqrt(gain / t_train) if gain > 0 else None
    # A trained network serves every later pricing of the same product: the
    # number of 1 bp pricings whose time saving pays for the training.
    out["break_even_pricings_1bp"] = t_train / gain if gain > 0 else None
    return out


def _line(args, metric, value, unit, ms, dtype, config, roofline, higher_is_better=True,
          **extra):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
         "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": higher_is_better,
         "scaling": "weak",
         "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config,
         "roofline": roofline}
    d.update(extra)
    return d


# HBM bytes per launch from rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE x 1 (KiB;
# the factors are what the counters read for a 1 GiB copy), for the kernels
# and launch shapes the profiles under profiles/ name; None where a kernel
# has no such measurement.
TRAFFIC_BYTES = {
    "gbm_path_kernel<float, asian|geo|uo, log-Euler>": 1.054e6,   # 2^24 paths x 252 steps
    "basket_kernel<8, bf16>": 2.595e6,                          # 2^20 paths x 100 steps
    "heston_adjoint_kernel<float, full, asian>": 2.261e6,       # 2^22 paths x 256 steps
    "lsm_update_kernel<2, 2, 1>": 3.660e8,                      # 2^24 paths, mean of 8 dates
}


def _alu_roofline(slots_per_unit, units, kernel_ms, kernel):
    achieved = slots_per_unit * units / (kernel_ms * 1e-3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_SLOTS / 1e12,
            "unit": "Tslot/s", "frac": achieved / ALU_PEAK_SLOTS,
            "traffic": TRAFFIC_BYTES.get(kernel), "slots_per_unit": slots_per_unit,
            "kernel": kernel}


def _repeat(args, torch, fn):
    """W warm-up steps, continued (up to 200 more) until 0.25 s have passed:
    the GPU's clocks ramp up over the first few tens of ms of work, and the
    timed steps are meant to run at steady clocks. Then the timed steps.
    Python's garbage collector is paused meanwhile (as timeit does): a full
    collection in a process holding torch takes tens of ms."""
    import gc
    gc_was_on = gc.isenabled()
    gc.disable()
    try:
        return _repeat_body(args, torch, fn)
    finally:
        if gc_was_on:
            gc.enable()


def _repeat_body(args, torch, fn):
    t0 = time.perf_counter()
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    extra = 0
    while args.warmup > 0 and time.perf_counter() - t0 < 0.25 and extra < 200:
        fn()
        torch.cuda.synchronize()
        extra += 1
    outs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outs.append(fn())
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / args.steps, outs


def gbm_time_to_1bp(ctx, mc, synth, torch):
    """Time to a standard error of 1 bp of the price for the estimators of the
    default workload's payoffs: the arithmetic Asian with and without the
    geometric-Asian control variate, and the up-and-out barrier. Each: a
    2^20-path pilot on stream tag 1 sizes N* = (s / (1e-4 p))^2, then one
    run of N* paths on tag 0; both are timed (the control variate's own
    coefficient pilot is part of its run; median of three pairs after an
    untimed one, see _pilot_then_run)."""
    c = synth.ASIAN_BARRIER
    n = c["n_steps"]
    model = mc.Model(kind=mc.MC_GBM, S0=c["S0"], r=c["r"], T=c["T"], sigma=c["sigma"])
    out = {"workload": f"GBM, {n} steps; target SE = 1e-4 x price"}
    for name, f in (("asian_geo_cv", mc.Payoff(mc.MC_ASIAN_ARITH_CALL, c["K"],
                                               cv=mc.MC_CV_GEO_ASIAN)),
                    ("asian_plain", mc.Payoff(mc.MC_ASIAN_ARITH_CALL, c["K"])),
                    ("uo_barrier", mc.Payoff(mc.MC_UO_BARRIER_CALL, c["K"], B=c["B"]))):
        pil, t_pil, N, run, t_run, totals = _pilot_then_run(
            torch, lambda: mc.mc_price(ctx, model, f, 1 << 20, n, synth.SEED,
                                       mc.Options(stream_tag=1)),
            lambda N: mc.mc_price(ctx, model, f, N, n, synth.SEED))
        out[name] = {"pilot_s": t_pil, "n_paths": N, "run_s": t_run, "total_s": t_pil + t_run,
                     "totals_s": totals, "price": run["price"], "std_err": run["std_err"],
                     "kernel_ms": run["kernel_ms"]}
    out["cv_speedup"] = out["asian_plain"]["total_s"] / out["asian_geo_cv"]["total_s"]
    return out


def run_asian_barrier(args, ctx, mc, synth, torch):
    c = synth.ASIAN_BARRIER
    N, n = c["n_paths"], c["n_steps"]
    model = mc.Model(kind=mc.MC_GBM, S0=c["S0"], r=c["r"], T=c["T"], sigma=c["sigma"])
    # A step is one whole pricing: the control-variate coefficient comes from
    # the step's own paths (in sample), so no pilot runs before or inside it.
    insample = mc.Options(pilot_paths=mc.MC_PILOT_IN_SAMPLE)
    payoffs = [mc.Payoff(mc.MC_ASIAN_ARITH_CALL, c["K"], cv=mc.MC_CV_GEO_ASIAN),
               mc.Payoff(mc.MC_UO_BARRIER_CALL, c["K"], B=c["B"]),
               mc.Payoff(mc.MC_ASIAN_GEO_CALL, c["K"])]
    step = mc.PreparedPriceMulti(ctx, model, payoffs, N, n, synth.SEED, insample)
    ms, outs = _repeat(args, torch, lambda: step()[0].kernel_ms)
    k_ms = sum(outs) / len(outs)
    res = step.results()
    line = _line(args, "path-steps/s", N * n / (ms * 1e-3), "path-steps/s", ms, "f32",
                 {"workload": "GBM arithmetic-Asian (geometric CV) + up-and-out barrier (B=130) "
                              "+ geometric Asian on the same paths, 2^24 paths x 252 log-Euler "
                              "steps, FP32 state, FP64 reduction, Philox4x32-10",
                  "n_paths": N, "n_steps": n},
                 _alu_roofline(SLOTS_ASIAN_BARRIER, N * n, k_ms,
                               "gbm_path_kernel<float, asian|geo|uo, log-Euler>"),
                 kernel_ms=k_ms,
                 prices={"asian_cv": res[0]["price"], "asian_cv_se": res[0]["std_err"],
                         "asian_plain": res[0]["plain_price"],
                         "asian_plain_se": res[0]["plain_std_err"],
                         "uo": res[1]["price"], "uo_se": res[1]["std_err"],
                         "geo": res[2]["price"], "geo_se": res[2]["std_err"],
                         "cv_beta": res[0]["cv_beta"], "vrf": res[0]["vrf"]})
    # Outside the timed region: the same paths with FP64 state, each FP32
    # price's distance from it in standard errors, and the geometric Asian
    # against its closed form.
    r64 = mc.mc_price_multi(ctx, model, payoffs, N, n, synth.SEED,
                            mc.Options(prec=mc.MC_FP64, pilot_paths=mc.MC_PILOT_IN_SAMPLE))
    pairs = (("asian_cv", res[0]["price"], r64[0]["price"], r64[0]["std_err"]),
             ("asian_plain", res[0]["plain_price"], r64[0]["plain_price"],
              r64[0]["plain_std_err"]),
             ("uo", res[1]["price"], r64[1]["price"], r64[1]["std_err"]),
             ("geo", res[2]["price"], r64[2]["price"], r64[2]["std_err"]))
    line["precision_check"] = {"fp64": {k: b for k, _, b, _ in pairs},
                               "diff_se": {k: (a - b) / se for k, a, b, se in pairs},
                               "rel_diff": {k: a / b - 1.0 for k, a, b, _ in pairs}}
    cg = _geo_asian_closed_form(c, n)
    line["closed_form"] = {"geo": cg, "geo_z": (res[2]["price"] - cg) / res[2]["std_err"]}
    if not args.no_time_to_1bp:
        line["time_to_1bp"] = time_to_1bp(ctx, mc, synth, torch, hedge_every=args.hedge_every,
                                          adam_steps=args.adam_steps)
        line["gbm_time_to_1bp"] = gbm_time_to_1bp(ctx, mc, synth, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c)
    return line


def run_european(args, ctx, mc, synth, torch):
    c = synth.EURO
    N, n = c["n_paths"], c["n_steps"]
    model = mc.Model(kind=mc.MC_GBM, S0=c["S0"], r=c["r"], T=c["T"], sigma=c["sigma"])
    f = mc.Payoff(mc.MC_EURO_CALL, c["K"])
    o = mc.Options(prec=mc.MC_FP64, greeks=mc.MC_GREEK_DELTA | mc.MC_GREEK_VEGA)
    ms, outs = _repeat(args, torch, lambda: mc.mc_price(ctx, model, f, N, n, synth.SEED, o))
    r = outs[-1]
    k_ms = sum(x["kernel_ms"] for x in outs) / len(outs)
    return _line(args, "path-steps/s", N * n / (ms * 1e-3), "path-steps/s", ms, "f64",
                 {"workload": "European call, GBM log-Euler, 64 steps, 2^18 paths, FP64, "
                              "pathwise delta and vega", "n_paths": N, "n_steps": n},
                 {"bound": "alu", "achieved": None, "peak": 78.6, "unit": "TFLOP/s (FP64)",
                  "frac": None, "traffic": None,
                  "note": "FP64 transcendentals go through library code; not modelled"},
                 kernel_ms=k_ms, prices={"price": r["price"], "se": r["std_err"],
                                         "delta": r["delta"], "vega": r["vega"]},
                 black_scholes=_bs_check(c, r))


def _geo_asian_closed_form(c, n):
    """Discrete geometric-Asian call on the fixings t_i = i T / n, i = 1..n.
    Under GBM ln G is normal with mean ln S0 + (r - s^2/2) T (n + 1) / (2 n)
    and variance s^2 T (n + 1)(2 n + 1) / (6 n^2), so the price is a
    lognormal call on G."""
    S, K, rr, s, T = c["S0"], c["K"], c["r"], c["sigma"], c["T"]
    m = math.log(S) + (rr - 0.5 * s * s) * T * (n + 1) / (2.0 * n)
    v = s * s * T * (n + 1) * (2 * n + 1) / (6.0 * n * n)
    d2 = (m - math.log(K)) / math.sqrt(v)
    d1 = d2 + math.sqrt(v)
    N = lambda x: 0.5 * (1.0 + math.erf(x / math.sqrt(2.0)))  # noqa: E731
    return math.exp(-rr * T) * (math.exp(m + 0.5 * v) * N(d1) - K * N(d2))


def _bs_check(c, r):
    """Black-Scholes price, delta and vega of the European call and the
    estimates' distance from them in standard errors (log-Euler is exact in
    law, so only Monte Carlo error separates them)."""
    S, K, rr, s, T = c["S0"], c["K"], c["r"], c["sigma"], c["T"]
    d1 = (math.log(S / K) + (rr + 0.5 * s * s) * T) / (s * math.sqrt(T))
    d2 = d1 - s * math.sqrt(T)
    N = lambda x: 0.5 * (1.0 + math.erf(x / math.sqrt(2.0)))  # noqa: E731
    price = S * N(d1) - K * math.exp(-rr * T) * N(d2)
    delta = N(d1)
    vega = S * math.sqrt(T) * math.exp(-0.5 * d1 * d1) / math.sqrt(2.0 * math.pi)
    return {"price": price, "delta": delta, "vega": vega,
            "price_z": (r["price"] - price) / r["std_err"],
            "delta_z": (r["delta"] - delta) / r["delta_se"],
            "vega_z": (r["vega"] - vega) / r["vega_se"]}


def run_basket(args, ctx, mc, synth, torch):
    c = synth.BASKET
    N, n, d = c["n_paths"], c["n_steps"], c["d"]
    sigma, corr, _ = synth.basket_market(d)
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=[c["S0"]] * d, r=c["r"], T=c["T"], sigma=sigma,
                     corr=corr)
    prec = {"fp32": mc.MC_FP32, "bf16": mc.MC_BF16_GEMM, "fp16": mc.MC_FP16_GEMM,
            "bf16x2": mc.MC_BF16X2_GEMM}[args.prec]
    f = mc.Payoff(mc.MC_BASKET_CALL, c["K"])
    o = mc.Options(prec=prec, greeks=mc.MC_GREEK_DELTA)
    ms, outs = _repeat(args, torch, lambda: mc.mc_price(ctx, model, f, N, n, synth.SEED, o))
    r = outs[-1]
    k_ms = sum(x["kernel_ms"] for x in outs) / len(outs)
    # MFMA work issued: lower-triangular 32x16 blocks per 32-path tile.
    nd = (d + 31) // 32
    blocks = sum(2 * nb + 2 for nb in range(nd))
    flops = (N // 32) * n * blocks * 32 * 32 * 16 * 2 * (2 if args.prec == "bf16x2" else 1)
    roof = _alu_roofline(SLOTS_ASSET_STEP, N * n * d, k_ms, f"basket_kernel<8, {args.prec}>")
    roof["mfma_tflops"] = flops / (k_ms * 1e-3) / 1e12
    roof["mfma_frac"] = flops / (k_ms * 1e-3) / MFMA_PEAK[args.prec]
    if args.prec != "fp32":
        # VALU issue and matrix-core time add up on a SIMD: the kernel against
        # their sum.
        n_mfma = (N // 32) * n * blocks * (2 if args.prec == "bf16x2" else 1)
        roof["mfma_share"] = _mfma_share(n_mfma, k_ms)
        roof["valu_plus_mfma_frac"] = roof["frac"] + roof["mfma_share"]
    extra = {}
    if prec != mc.MC_FP32:
        # The rounding of the reduced-precision product at the full size: the
        # same paths with FP32 products (within 2e-5 of the FP64 oracle),
        # outside the timed region.
        ref = mc.mc_price(ctx, model, f, N, n, synth.SEED,
                          mc.Options(prec=mc.MC_FP32, greeks=mc.MC_GREEK_DELTA))
        extra["precision_check"] = {
            "fp32_price": ref["price"], "fp32_delta0": ref["delta"],
            "price_diff_se": (r["price"] - ref["price"]) / ref["std_err"],
            "delta0_diff_se": (r["delta"] - ref["delta"]) / ref["delta_se"],
            "price_rel_diff": r["price"] / ref["price"] - 1.0}
    return _line(args, "asset-path-steps/s", N * n * d / (ms * 1e-3), "asset-path-steps/s", ms,
                 args.prec,
                 {"workload": f"basket call, d = {d} correlated GBM, {n} steps, 2^20 paths, "
                              f"per-step Z L^T on MFMA ({args.prec})", "n_paths": N,
                  "n_steps": n, "d": d},
                 roof, kernel_ms=k_ms,
                 prices={"price": r["price"], "se": r["std_err"], "delta0": r["delta"],
                         "delta0_se": r["delta_se"]}, **extra)


def run_mlmc_basket(args, ctx, mc, synth, torch):
    """Time to a standard error of 1 bp of the price on the d = 256 basket:
    plain FP32 Monte Carlo against the two-level estimator whose level 0
    runs the BF16 matrix product and whose level 1 corrects it to FP32 on
    shared paths (the low-precision companion estimator with a reference-
    precision correction). Each side: a 2^18-path pilot (stream tag 1, and
    1 + 16 for the pilot's correction level) sizes the main run (tag 0;
    the multilevel path counts from mc_mlmc_allocate with the pilot's level
    variances and measured per-path device times); pilot and run are timed."""
    c = synth.BASKET
    n, d = c["n_steps"], c["d"]
    sigma, corr, _ = synth.basket_market(d)
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=[c["S0"]] * d, r=c["r"], T=c["T"], sigma=sigma,
                     corr=corr)
    f = mc.Payoff(mc.MC_BASKET_CALL, c["K"])
    pilot = 1 << 18
    pil, t_pil = _timed(torch, lambda: mc.mc_price(ctx, model, f, pilot, n, synth.SEED,
                                                   mc.Options(prec=mc.MC_FP32, stream_tag=1)))
    N_plain = _paths_for(1e-4 * pil["price"], math.sqrt(pil["variance"]))
    run, t_run = _timed(torch, lambda: mc.mc_price(ctx, model, f, N_plain, n, synth.SEED,
                                                   mc.Options(prec=mc.MC_FP32)))
    plain = {"pilot_s": t_pil, "n_paths": N_plain, "run_s": t_run, "total_s": t_pil + t_run,
             "price": run["price"], "std_err": run["std_err"], "kernel_ms": run["kernel_ms"]}
    lp = [mc.Level(n, mc.MC_BF16_GEMM, pilot), mc.Level(n, mc.MC_FP32, pilot)]
    mp, t_mp = _timed(torch, lambda: mc.mc_price_mlmc(ctx, model, f, lp, synth.SEED,
                                                      mc.Options(stream_tag=1)))
    var = [lv["variance"] for lv in mp["levels"]]
    cost = [lv["kernel_ms"] / lv["n_paths"] for lv in mp["levels"]]
    N = mc.mc_mlmc_allocate(var, cost, 1e-4 * mp["price"])
    levels = [mc.Level(n, mc.MC_BF16_GEMM, N[0]), mc.Level(n, mc.MC_FP32, N[1])]
    mr, t_mr = _timed(torch, lambda: mc.mc_price_mlmc(ctx, model, f, levels, synth.SEED))
    l0, l1 = mr["levels"]
    mlmc = {"pilot_s": t_mp, "pilot_var": var, "pilot_cost_ms_per_path": cost, "n_paths": N,
            "run_s": t_mr, "total_s": t_mp + t_mr, "price": mr["price"],
            "std_err": mr["std_err"], "level_kernel_ms": [l0["kernel_ms"], l1["kernel_ms"]],
            "bf16_bias": l1["mean"], "bf16_bias_se": math.sqrt(l1["variance"] / l1["n_paths"]),
            "level0_price": l0["mean"]}
    k_ms = l0["kernel_ms"]
    roof = _alu_roofline(SLOTS_ASSET_STEP, N[0] * n * d, k_ms, "basket_kernel<8, bf16>")
    return _line(args, "time to 1bp SE", mlmc["total_s"], "s", mlmc["total_s"] * 1e3, "bf16",
                 {"workload": f"basket call, d = {d} correlated GBM, {n} steps; target SE = "
                              "1e-4 x price; BF16 level + FP32 correction level vs plain FP32",
                  "n_steps": n, "d": d},
                 roof, higher_is_better=False,
                 time_to_1bp={"plain_fp32": plain, "mlmc_bf16_fp32": mlmc,
                              "speedup": plain["total_s"] / mlmc["total_s"]})


def run_qmc_basket(args, ctx, mc, synth, torch):
    """Sobol' randomised QMC against Philox Monte Carlo on a 16-asset basket
    call in one step (the setting of the Sobol' experiment): 16 replicates of
    2^16 points against one Monte Carlo run of 2^20 paths; standard errors,
    device times and the efficiency gain (SE^2 x time ratio). FP32 matrix
    products by default: BF16 moves this 16-asset price by about 4e-4
    relative, several times the QMC standard error."""
    d = 16
    sigma, corr, _ = synth.basket_market(d)
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=[100.0] * d, r=0.05, T=1.0, sigma=sigma,
                     corr=corr)
    f = mc.Payoff(mc.MC_BASKET_CALL, 100.0)
    prec = {"fp32": mc.MC_FP32, "bf16": mc.MC_BF16_GEMM, "fp16": mc.MC_FP16_GEMM}.get(
        args.prec, mc.MC_FP32)
    R, NQ = 16, 1 << 16
    ms, outs = _repeat(args, torch, lambda: mc.mc_price_qmc(ctx, model, f, NQ, 1, synth.SEED, R,
                                                             mc.Options(prec=prec)))
    q = outs[-1]
    mcr = mc.mc_price(ctx, model, f, R * NQ, 1, synth.SEED, mc.Options(prec=prec))
    gain = (mcr["std_err"] ** 2 * mcr["kernel_ms"]) / (q["std_err"] ** 2 * q["kernel_ms"])
    k_ms = q["kernel_ms"] / R
    roof = _alu_roofline(SLOTS_ASSET_STEP, NQ * d, k_ms, f"basket_kernel<1, {args.prec}, qmc>")

    # The paper's only printed timing (Sec. VI-D): median wall time of 100
    # calls pricing this basket call on 8192 samples, for pseudo-random MC
    # and for Sobol' points. Context from other hardware, not a target.
    def median_ms(fn, trials=100):
        ts = []
        for _ in range(trials):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts) * 1e3
    ctx_mc = median_ms(lambda: mc.mc_price(ctx, model, f, 8192, 1, synth.SEED, mc.Options(prec=prec)))
    ctx_qmc = median_ms(lambda: mc.mc_price_qmc(ctx, model, f, 8192, 1, synth.SEED, 1,
                                                mc.Options(prec=prec)))
    return _line(args, "paths/s", R * NQ / (ms * 1e-3), "paths/s", ms, args.prec,
                 {"workload": "basket call, d = 16, one step, randomised Sobol' QMC "
                              "(16 digital shifts x 2^16 points) vs Philox MC (2^20 paths)",
                  "n_points": NQ, "replicates": R, "d": d},
                 roof, kernel_ms=q["kernel_ms"],
                 qmc={"price": q["price"], "std_err": q["std_err"],
                      "geo_price": q["geo_price"], "geo_std_err": q["geo_std_err"],
                      "mc_price": mcr["price"], "mc_std_err": mcr["std_err"],
                      "mc_kernel_ms": mcr["kernel_ms"], "variance_ratio":
                      (mcr["std_err"] / q["std_err"]) ** 2, "efficiency_gain": gain},
                 paper_context={"samples": 8192, "median_ms_mc": ctx_mc, "median_ms_qmc": ctx_qmc,
                                "paper_ms_mc": 1.40, "paper_ms_qmc": 1.15,
                                "note": "paper: Cloud TPU, Threefry and Sobol', median of 100 "
                                        "calls including the cloud round trip; here: one MI355X, "
                                        "Philox and Sobol' (one digital shift), median of 100 "
                                        "blocking library calls"})


RISK_STRIKES = [0.9, 0.95, 1.0, 1.05, 1.1]
RISK_QTY = [1.0, -2.0, 1.5, -1.0, 0.5]


def run_risk(args, ctx, mc, synth, torch):
    """VaR_0.95 and CVaR_0.95 of a portfolio of 5 calls on each of the
    basket's 256 assets (1280 instruments) over a one-year horizon in 100
    steps, 2^20 scenarios under real-world drifts; the matrix-product
    precision of --prec, with the FP32 values beside it for the bias."""
    c = synth.BASKET
    N, n, d = c["n_paths"], c["n_steps"], c["d"]
    sigma, corr, _ = synth.basket_market(d)
    S0 = [c["S0"]] * d
    mu = [0.02 + 0.08 * a / (d - 1) for a in range(d)]
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=S0, r=c["r"], T=c["T"], sigma=sigma, corr=corr)
    prec = {"fp32": mc.MC_FP32, "bf16": mc.MC_BF16_GEMM, "fp16": mc.MC_FP16_GEMM}.get(
        args.prec, mc.MC_BF16_GEMM)

    def go(p):
        return mc.mc_risk(ctx, model, RISK_STRIKES, RISK_QTY, 0.95, N, n, synth.SEED, mu=mu,
                          opts=mc.Options(prec=p))
    ms, outs = _repeat(args, torch, lambda: go(prec))
    r = outs[-1]
    ref = go(mc.MC_FP32)
    k_ms = sum(x["kernel_ms"] for x in outs) / len(outs)
    s_ms = sum(x["select_ms"] for x in outs) / len(outs)
    roof = _alu_roofline(SLOTS_ASSET_STEP, N * n * d, k_ms, f"basket_kernel<8, {args.prec}, port>")
    return _line(args, "scenario-asset-steps/s", N * n * d / (ms * 1e-3), "asset-path-steps/s",
                 ms, args.prec,
                 {"workload": f"VaR/CVaR 0.95 of 5 calls on each of {d} correlated GBM assets "
                              f"({5 * d} instruments), 1-year horizon in {n} steps, 2^20 "
                              f"scenarios, real-world drifts", "n_paths": N, "n_steps": n,
                  "d": d},
                 roof, kernel_ms=k_ms, select_ms=s_ms,
                 risk={"var": r["var"], "cvar": r["cvar"], "pnl_mean": r["pnl_mean"],
                       "premium": r["premium"], "var_fp32": ref["var"],
                       "cvar_fp32": ref["cvar"],
                       "var_rel_diff": r["var"] / ref["var"] - 1.0,
                       "cvar_rel_diff": r["cvar"] / ref["cvar"] - 1.0})


def run_heston_adjoint(args, ctx, mc, synth, torch):
    import numpy as np
    H = synth.HESTON
    N, n = H["n_paths"], H["n_steps"]
    model = _heston_model(mc, synth)
    f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, H["K"])
    o = mc.Options(greeks=mc.MC_GREEK_DELTA | mc.MC_GREEK_VEGA)
    ms, outs = _repeat(args, torch, lambda: mc.mc_price(ctx, model, f, N, n, synth.SEED, o))
    r = outs[-1]
    k_ms = sum(x["kernel_ms"] for x in outs) / len(outs)
    per_step = 2 * SLOTS_HESTON + SLOTS_HESTON_REVERSE   # forward, recompute, reverse
    # Beside it: the price alone (forward kernel only) on the same paths, and
    # central differences on common random numbers (h = 1e-3 relative, FP64
    # bumped pairs) on 2^20 of them as the independent check of the greeks.
    fwd = [mc.mc_price(ctx, model, f, N, n, synth.SEED)["kernel_ms"] for _ in range(3)]
    # The same greeks in forward mode: tangents carried beside the state, no
    # checkpoints, no reverse sweep.
    to = mc.Options(greeks=mc.MC_GREEK_DELTA | mc.MC_GREEK_VEGA,
                    greeks_method=mc.MC_GREEKS_TANGENT)
    tan = [mc.mc_price(ctx, model, f, N, n, synth.SEED, to) for _ in range(3)]
    t_ms = min(x["kernel_ms"] for x in tan)
    # The same paths with FP64 state (forward tangents in FP64): the FP32
    # adjoint's price and greeks against them, in standard errors of each
    # estimate and of the per-path differences. The FP32 d/dv0 sits about half
    # a standard error off; the bound stated beside it: the mean per-path
    # difference is within 4 standard errors of the differences, and without
    # the 100 largest per-path differences the rest is within 0.01 standard
    # errors of the greek (the difference lives on the few paths whose
    # variance reaches zero within FP32 resolution).
    r64 = mc.mc_price(ctx, model, f, N, n, synth.SEED,
                      mc.Options(prec=mc.MC_FP64, greeks=mc.MC_GREEK_DELTA | mc.MC_GREEK_VEGA,
                                 greeks_method=mc.MC_GREEKS_TANGENT, path_values=True))
    pv32 = mc.mc_greeks_adjoint(ctx, model, f, N, n, synth.SEED,
                                mc.Options(path_values=True))["path_values"]
    per_path = {}
    for c, name in ((0, "price"), (1, "delta"), (2, "dv0")):
        d = pv32[:, c] - r64["path_values"][:, c]
        se_g = r64["path_values"][:, c].std(ddof=1) / math.sqrt(N)
        top = np.argsort(np.abs(d))[::-1][:100]
        per_path[name] = {"mean_diff_se_of_diff": float(d.mean() / (d.std(ddof=1) / math.sqrt(N))),
                          "rest_without_top100_se": float((d.sum() - d[top].sum()) / N / se_g),
                          "max_abs_diff": float(np.abs(d).max())}
    per_path["bound"] = ("FP32 price and delta within 0.1 SE of FP64 state; d/dv0 not: its "
                         "mean per-path difference within 4 SE of the differences, and within "
                         "0.01 SE of the greek without the 100 largest per-path differences")
    del pv32
    fd = mc.mc_price(ctx, model, f, 1 << 20, n, synth.SEED,
                     mc.Options(greeks=mc.MC_GREEK_DELTA | mc.MC_GREEK_VEGA,
                                greeks_method=mc.MC_GREEKS_FD_CRN))

    def z(a, sa, b, sb):
        return (a - b) / math.hypot(sa, sb)
    return _line(args, "path-steps/s", N * n / (ms * 1e-3), "path-steps/s", ms, "f32",
                 {"workload": "Heston arithmetic-Asian call, full-truncation Euler, 256 steps, "
                              "2^22 paths, price + pathwise delta and d/dv0 by the checkpointed "
                              "adjoint (every 16 steps)", "n_paths": N, "n_steps": n},
                 _alu_roofline(per_step, N * n, k_ms, "heston_adjoint_kernel<float, full, asian>"),
                 kernel_ms=k_ms,
                 forward_only={"kernel_ms": min(fwd), "path_steps_per_s": N * n / (min(fwd) * 1e-3)},
                 forward_tangent={"kernel_ms": t_ms, "path_steps_per_s": N * n / (t_ms * 1e-3),
                                  "delta": tan[-1]["delta"], "dv0": tan[-1]["vega"]},
                 prices={"price": r["price"], "se": r["std_err"], "delta": r["delta"],
                         "delta_se": r["delta_se"], "dv0": r["vega"], "dv0_se": r["vega_se"]},
                 precision_check={
                     "fp64": {"price": r64["price"], "delta": r64["delta"], "dv0": r64["vega"]},
                     "diff_se": {"price": (r["price"] - r64["price"]) / r64["std_err"],
                                 "delta": (r["delta"] - r64["delta"]) / r64["delta_se"],
                                 "dv0": (r["vega"] - r64["vega"]) / r64["vega_se"]},
                     "rel_diff": {"price": r["price"] / r64["price"] - 1.0,
                                  "delta": r["delta"] / r64["delta"] - 1.0,
                                  "dv0": r["vega"] / r64["vega"] - 1.0},
                     "per_path": per_path},
                 fd_check={"n_paths": 1 << 20, "delta": fd["delta"], "delta_se": fd["delta_se"],
                           "dv0": fd["vega"], "dv0_se": fd["vega_se"],
                           "delta_z": z(r["delta"], r["delta_se"], fd["delta"], fd["delta_se"]),
                           "dv0_z": z(r["vega"], r["vega_se"], fd["vega"], fd["vega_se"])})


def run_learned_cv(args, ctx, mc, synth, torch):
    out = time_to_1bp(ctx, mc, synth, torch, hedge_every=args.hedge_every,
                      adam_steps=args.adam_steps)
    n = synth.HESTON["n_steps"]
    cv = out["learned_cv_bf16"]
    m = args.hedge_every
    # Per date and path (two 32-path network passes per wave of 64 paths):
    # 64 tanh of layer 1, 64 sigmoid-form activations of layer 2, 64 FMAs of
    # layer 3 and 8 feature operations.
    per_step = SLOTS_HESTON + (64 * SLOTS_TANH + 64 * SLOTS_SIGM + slots(fp32=64 + 8)) / m
    roof = _alu_roofline(per_step, cv["n_paths"] * n, cv["kernel_ms"], "cv_eval_kernel<bf16>")
    # Two network passes (2 + 8 MFMAs each) per wave of 64 paths per date.
    n_mfma = -(-cv["n_paths"] // 64) * -(-n // m) * 20
    roof["mfma_share"] = _mfma_share(n_mfma, cv["kernel_ms"])
    roof["valu_plus_mfma_frac"] = roof["frac"] + roof["mfma_share"]
    return _line(args, "time to 1bp SE", cv["total_s"], "s", cv["total_s"] * 1e3, "bf16",
                 {"workload": out["workload"] + f", learned CV rebalanced every {m} steps",
                  "n_steps": n},
                 roof, higher_is_better=False, time_to_1bp=out)


# Bermudan call on the maximum of two assets (the LSM experiment of Sec. VI-C):
# independent assets S0 = 100, sigma = 0.2, dividend yield 0.1, r = 0.05,
# K = 100, T = 3, 9 exercise dates; 2^24 in-sample and 2^24 fresh paths.
LSM = dict(S0=[100.0, 100.0], sigma=[0.2, 0.2], r=0.05, q=0.10, T=3.0, K=100.0, n_dates=9,
           degree=2, n_paths=1 << 24, n_oos=1 << 24)
PAPER_LSM_PRICE = 13.90   # the true price the paper quotes for this option


def _lsm_update_bytes(N, M, d):
    """Algorithmic HBM bytes of the M-1 update kernels: every date reads the
    states of its own date and of the previous one (FP32, d assets) and the
    cash flow; date 1 reads only its own states. Cash-flow writes (only the
    exercising paths) are not counted."""
    return N * ((M - 2) * (8 * d + 4) + (4 * d + 4))


def lsm_cpu_baseline(c, n_paths=1 << 20):
    """The FP64 oracle's Longstaff-Schwartz (in-sample regression and the
    out-of-sample estimate on as many fresh paths) on a sample of the paths."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    o = oracle.lsm(c["S0"], c["sigma"], np.eye(2), c["r"], c["q"], c["T"], 1, c["K"],
                   c["n_dates"], 1, c["degree"], n_paths, 1234)
    oracle.lsm_oos(c["S0"], c["sigma"], np.eye(2), c["r"], c["q"], c["T"], 1, c["K"],
                   c["n_dates"], 1, c["degree"], o["beta"], n_paths, 1234, tag=7)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_paths / dt, "unit": "paths/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": f"{n_paths} of {c['n_paths']} in-sample paths plus {n_paths} fresh paths "
                      f"(FP64 oracle), {dt:.1f} s"}


def run_lsm(args, ctx, mc, synth, torch):
    """Longstaff-Schwartz price of the two-asset Bermudan max-call: path
    simulation with stored exercise-date states, 8 chained FP64 regressions
    and the out-of-sample estimate, one mc_price_lsm call per step."""
    import numpy as np
    c = LSM
    N, M, d = c["n_paths"], c["n_dates"], 2
    model = mc.Model(kind=mc.MC_GBM_BASKET, S0=c["S0"], r=c["r"], T=c["T"], sigma=c["sigma"],
                     corr=np.eye(2))
    spec = mc.LsmSpec(payoff=mc.MC_LSM_MAX_CALL, K=c["K"], dividend=c["q"], n_dates=M,
                      steps_per_date=1, degree=c["degree"], n_paths_oos=c["n_oos"])
    ms, outs = _repeat(args, torch, lambda: mc.mc_price_lsm(ctx, model, spec, N, synth.SEED))
    r = outs[-1]

    def avg(k):
        return sum(x[k] for x in outs) / len(outs)
    upd = avg("update_ms")
    kernel = "lsm_update_kernel<2, 2, 1>"
    achieved = _lsm_update_bytes(N, M, d) / (upd * 1e-3)
    roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "traffic": TRAFFIC_BYTES.get(kernel), "kernel": kernel,
            "bytes_per_launch": _lsm_update_bytes(N, M, d) / (M - 1), "launches": M - 1}
    line = _line(args, "paths/s", N / (ms * 1e-3), "paths/s", ms, "f32",
                 {"workload": "Bermudan call on the max of two independent GBM assets (S0 100, "
                              "sigma 0.2, dividend yield 0.1, r 0.05, K 100, T 3, 9 dates), "
                              "Longstaff-Schwartz with degree-2 monomials and the payoff, "
                              "2^24 in-sample + 2^24 out-of-sample paths", "n_paths": N,
                  "n_paths_oos": c["n_oos"], "n_dates": M, "d": d},
                 roof, sim_ms=avg("sim_ms"), regress_ms=avg("regress_ms"), update_ms=upd,
                 oos_ms=avg("oos_ms"),
                 lsm={"price": r["price"], "std_err": r["std_err"], "price_oos": r["price_oos"],
                      "std_err_oos": r["std_err_oos"], "european": r["european"],
                      "european_se": r["european_se"], "paper_true_price": PAPER_LSM_PRICE})
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = lsm_cpu_baseline(c)
    return line


WORKLOADS = {"asian_barrier": run_asian_barrier, "european": run_european, "basket": run_basket,
             "heston_adjoint": run_heston_adjoint, "learned_cv": run_learned_cv,
             "mlmc_basket": run_mlmc_basket, "risk": run_risk, "qmc_basket": run_qmc_basket,
             "lsm": run_lsm}


# ---- the oracle beside each workload (bounded samples on the host cores) ----
def _cpu_european(line, synth):
    import oracle
    c = synth.EURO
    n = c["n_steps"]
    N, dt = _oracle_sample(lambda k: oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"],
                                                1e300, n, k, 1234), 1 << 12, c["n_paths"])
    return _cpu_entry(N * n / dt, "path-steps/s",
                      f"{N} of {c['n_paths']} paths x {n} steps, FP64 GBM oracle (price and "
                      f"pathwise tangents among its channels), {dt:.1f} s")


def _basket_rate(synth, c, probe=1 << 8):
    import numpy as np
    import oracle
    n, d = c["n_steps"], c["d"]
    sigma, L, w = _basket_oracle_inputs(synth, d)
    S0 = np.full(d, c["S0"])
    N, dt = _oracle_sample(lambda k: oracle.basket(S0, sigma, L, w, c["r"], c["T"], c["K"], n,
                                                   k, 1234), probe, c["n_paths"])
    return N, dt


def _cpu_basket(line, synth):
    c = synth.BASKET
    n, d = c["n_steps"], c["d"]
    N, dt = _basket_rate(synth, c)
    return _cpu_entry(N * n * d / dt, "asset-path-steps/s",
                      f"{N} of {c['n_paths']} paths x {n} steps x {d} assets, FP64 basket "
                      f"oracle (Z L^T as a plain triangular product), {dt:.1f} s")


def _cpu_mlmc_basket(line, synth):
    c = synth.BASKET
    n, d = c["n_steps"], c["d"]
    N, dt = _basket_rate(synth, c)
    n_plain = line["time_to_1bp"]["plain_fp32"]["n_paths"]
    return _cpu_entry(n_plain * dt / N, "s",
                      f"{N} basket paths ({n} steps x {d} assets, FP64 oracle) in {dt:.1f} s, "
                      f"projected to the {n_plain} paths of the plain estimator at SE = 1 bp",
                      sample_s=dt)


def _cpu_risk(line, synth):
    import numpy as np
    import oracle
    c = synth.BASKET
    n, d = c["n_steps"], c["d"]
    sigma, L, _ = _basket_oracle_inputs(synth, d)
    S0 = np.full(d, c["S0"])
    mu = [0.02 + 0.08 * a / (d - 1) for a in range(d)]

    def run(k):
        pnl = oracle.portfolio_pnl(S0, sigma, mu, L, RISK_STRIKES, RISK_QTY, c["r"], c["T"], n,
                                   k, 1234)
        oracle.var_cvar(pnl, 0.95)
    N, dt = _oracle_sample(run, 1 << 8, c["n_paths"])
    return _cpu_entry(N * n * d / dt, "asset-path-steps/s",
                      f"{N} of {c['n_paths']} scenarios x {n} steps x {d} assets, FP64 "
                      f"portfolio oracle and a sorted VaR/CVaR, {dt:.1f} s")


def _cpu_heston_adjoint(line, synth):
    import oracle
    H = synth.HESTON
    n = H["n_steps"]
    N, dt = _oracle_sample(lambda k: oracle.heston(
        H["S0"], H["v0"], H["kappa"], H["theta"], H["xi"], H["rho"], H["r"], H["T"], H["K"], n,
        k, 1234), 1 << 10, H["n_paths"])
    return _cpu_entry(N * n / dt, "path-steps/s",
                      f"{N} of {H['n_paths']} paths x {n} steps, FP64 Heston oracle (price "
                      f"and forward-mode pathwise delta and d/dv0), {dt:.1f} s")


def _cpu_learned_cv(line, synth):
    import oracle
    H = synth.HESTON
    n = H["n_steps"]
    t1 = line["time_to_1bp"]
    N, dt = _oracle_sample(lambda k: oracle.heston(
        H["S0"], H["v0"], H["kappa"], H["theta"], H["xi"], H["rho"], H["r"], H["T"], H["K"], n,
        k, 1234), 1 << 10, 1 << 20, budget_s=6.0)
    m = t1["hedge_every"]
    th = synth.glorot_mlp()
    Nc, dtc = _oracle_sample(lambda k: oracle.heston_cv(H, n, th, k, 1234, m_every=m),
                             1 << 8, 1 << 20, budget_s=6.0)
    n_plain, n_cv = t1["plain_fp32"]["n_paths"], t1["learned_cv_bf16"]["n_paths"]
    return _cpu_entry(n_plain * dt / N, "s",
                      f"{N} Heston paths ({n} steps, FP64 oracle) in {dt:.1f} s, projected "
                      f"to the {n_plain} paths of the plain estimator at SE = 1 bp",
                      learned_cv_eval_s=n_cv * dtc / Nc,
                      learned_cv_sample=f"{Nc} paths of the FP64 hedge-network oracle "
                                        f"(rebalanced every {m} steps) in {dtc:.1f} s, "
                                        f"projected to the {n_cv} paths of the learned-CV "
                                        f"estimator; training excluded")


def _cpu_qmc_basket(line, synth):
    import numpy as np
    import oracle
    d = 16
    sigma, L, w = _basket_oracle_inputs(synth, d)
    S0 = np.full(d, 100.0)
    NQ, R = line["config"]["n_points"], line["config"]["replicates"]

    def run(k):
        for rep in range(R):
            oracle.basket_qmc(S0, sigma, L, w, 0.05, 1.0, 100.0, 1, k, 1234, rep)
    N, dt = _oracle_sample(run, NQ, NQ)
    return _cpu_entry(R * N / dt, "paths/s",
                      f"{N} of the {NQ} points of each of the {R} replicates (16-asset basket, "
                      f"one step, FP64 Sobol' oracle), {dt:.1f} s")


CPU_BASELINES = {
    "european": _cpu_european,
    "basket": _cpu_basket,
    "mlmc_basket": _cpu_mlmc_basket,
    "risk": _cpu_risk,
    "heston_adjoint": _cpu_heston_adjoint,
    "learned_cv": _cpu_learned_cv,
    "qmc_basket": _cpu_qmc_basket,
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=list(WORKLOADS), default="asian_barrier")
    ap.add_argument("--prec", choices=["fp32", "bf16", "fp16", "bf16x2"], default=None,
                    help="matrix-product precision (default: bf16 for basket and risk, fp32 "
                         "for qmc_basket, which refuses bf16: its standard error is below "
                         "the BF16 bias)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-1bp", action="store_true")
    ap.add_argument("--hedge-every", type=int, default=16)
    ap.add_argument("--adam-steps", type=int, default=None,
                    help="training steps of the hedge network in the time-to-1bp comparison "
                         "(default: the recipe's 2000)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; the path range shards "
                          "across GPUs by path_offset, but only --gpus 1 is measured"}))
        sys.exit(2)

    import torch
    import paper_1906_02818_amd as mc
    import synth

    ctx = mc.mc_create(0)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.prec is None:
        args.prec = "fp32" if args.workload == "qmc_basket" else "bf16"
    line = WORKLOADS[args.workload](args, ctx, mc, synth, torch)
    if (not args.no_cpu_baseline and "cpu_baseline" not in line
            and args.workload in CPU_BASELINES):
        line["cpu_baseline"] = CPU_BASELINES[args.workload](line, synth)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
