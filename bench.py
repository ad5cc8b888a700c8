"""Benchmark of the Monte Carlo path engine on one MI355X.

Workload: arithmetic-average Asian call (with the geometric-Asian control
variate) and discretely monitored up-and-out call (B = 130) priced on the
same 1-D GBM paths: S0 = K = 100, r = 0.03, sigma = 0.25, T = 1, 252
log-Euler steps, 2^24 paths, FP32 path state, FP64 cross-path reduction,
Philox4x32-10 seed 1234. One step of the benchmark is one full pricing pass:
the path kernel (random numbers, Euler-Maruyama steps, path functionals,
payoffs, block moments), the fixed-order final reduction and the read-back
of the moments. Inputs are parameters only, so nothing is staged from the
host in the timed region.

Prints one JSON line. `roofline` reports the path kernel against the ALU
issue peak (it reads and writes no HBM per step); `time_to_1bp` compares,
after the timed region, plain FP32 Monte Carlo with the learned control
variate (BF16 matrix products) on the Heston Asian call; `cpu_baseline`
times the FP64 oracle on a bounded sample of the benchmarked workload on the
host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz; the FP32 vector peak (157.3 TFLOP/s) is 128
# FMA lanes per clock per CU, the unit ("slot") of the ALU roofline.
N_CU, CLOCK_HZ, FMA_LANES_PER_CLK = 256, 2.4e9, 128
ALU_PEAK_SLOTS = N_CU * CLOCK_HZ * FMA_LANES_PER_CLK      # 7.86e13 slots/s

# Issue cost of each instruction class in FMA slots on gfx950: 2 wave64
# FMAs per clock per CU divided by the rate measured for that instruction by
# paper_1906_02818_amd/isa_rates.hip (profiles/isa_rates.txt).
COST_MUL64 = 3.7     # 32x32->64-bit product (v_mad_u64_u32)
COST_TRANS = 4.1     # v_exp / log / sin / cos / sqrt / rcp _f32
COST_INT = 0.56      # xor, shift, or, compare (gfx950 has no three-input xor)
COST_FP32 = 1.0      # add, mul, fma

# Algorithmic operations per path-step of the benchmarked workload (one
# normal per step):
#   Philox4x32-10: 10 rounds x (2 mul64 + 4 xor) per 4 normals
#   uniform: shift, or, sub per uniform, one uniform per normal
#   Box-Muller: log, sqrt, sin, cos and 3 mul per 2 normals
#   step: fma + add; Asian: exp2 + add; geometric: add; barrier: compare
SLOTS_PER_PATH_STEP = (5.0 * COST_MUL64 + 3.0 * COST_TRANS
                       + (10.0 + 2.0 + 1.0) * COST_INT
                       + (1.0 + 1.5 + 2.0 + 1.0 + 1.0) * COST_FP32)


def cpu_baseline(c, budget_s=12.0):
    """FP64 oracle on the host cores over a bounded sample of the workload."""
    import oracle
    n = c["n_steps"]
    t0 = time.perf_counter()
    probe = 1 << 12
    oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], c["B"], n, probe, 1234)
    dt = time.perf_counter() - t0
    n_paths = int(max(probe, min(c["n_paths"], probe * budget_s / max(dt, 1e-6))))
    n_paths = 1 << int(math.log2(n_paths))
    t0 = time.perf_counter()
    oracle.gbm(c["S0"], c["r"], c["sigma"], c["T"], c["K"], c["B"], n, n_paths, 1234)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_paths * n / dt, "unit": "path-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_paths} of {c['n_paths']} paths x {n} steps, all channels of the "
                      f"GBM oracle (FP64), {dt:.1f} s"}


def _paths_for(se_target, sigma):
    n = int(math.ceil((sigma / se_target) ** 2))
    return max(256, (n + 255) // 256 * 256)


def time_to_1bp(ctx, mc, synth, hedge_every=8, adam_steps=2000):
    """Time to a Heston-Asian price whose standard error is 1 bp of the price
    (1e-4 x price), plain FP32 Monte Carlo against the learned control
    variate with BF16 matrix products. Each estimator: a 2^20-path pilot on
    stream tag 1 sizes N* = (s / (1e-4 p))^2, then one run of N* paths on
    tag 0; both are timed. The hedge network is trained beforehand (2000
    Adam steps, minibatch 2^16 from a fixed 2^20-path set on tag 2); its
    training time is reported separately and added in `total_incl_train_s`.
    """
    import numpy as np
    import torch
    H = synth.HESTON
    cv = synth.LEARNED_CV
    n = H["n_steps"]
    model = mc.Model(kind=mc.MC_HESTON, S0=H["S0"], r=H["r"], T=H["T"], v0=H["v0"],
                     kappa=H["kappa"], theta=H["theta"], xi=H["xi"], rho=H["rho"])
    plain_f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, H["K"])
    cv_f = mc.Payoff(mc.MC_ASIAN_ARITH_CALL, H["K"], cv=mc.MC_CV_LEARNED)
    out = {"workload": f"Heston arithmetic-Asian call, {n} steps; target SE = 1e-4 x price",
           "hedge_every": hedge_every}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    # Plain FP32.
    pil, t_pil = timed(lambda: mc.mc_price(ctx, model, plain_f, 1 << 20, n, synth.SEED,
                                           mc.Options(stream_tag=1)))
    sig = math.sqrt(pil["variance"])
    N_plain = _paths_for(1e-4 * pil["price"], sig)
    run, t_run = timed(lambda: mc.mc_price(ctx, model, plain_f, N_plain, n, synth.SEED))
    out["plain_fp32"] = {"pilot_s": t_pil, "n_paths": N_plain, "run_s": t_run,
                         "total_s": t_pil + t_run, "price": run["price"],
                         "std_err": run["std_err"], "kernel_ms": run["kernel_ms"]}
    # Learned CV, BF16.
    th0 = synth.glorot_mlp()
    (w, log), t_train = timed(lambda: mc.mc_cv_train(
        ctx, model, cv_f, cv["n_train"], n, synth.SEED, th0, lr=cv["lr"], steps=adam_steps,
        batch=cv["batch"], hedge_every=hedge_every, prec=mc.MC_BF16_GEMM))
    opts = lambda tag: mc.Options(prec=mc.MC_BF16_GEMM, cv_weights=w, cv_hedge_every=hedge_every,
                                  cv_beta=1.0, stream_tag=tag)
    pil, t_pil = timed(lambda: mc.mc_price(ctx, model, cv_f, 1 << 20, n, synth.SEED, opts(1)))
    N_cv = _paths_for(1e-4 * pil["price"], math.sqrt(pil["variance"]))
    run, t_run = timed(lambda: mc.mc_price(ctx, model, cv_f, N_cv, n, synth.SEED, opts(0)))
    out["learned_cv_bf16"] = {"train_s": t_train, "adam_steps": adam_steps,
                              "loss_first": float(log[0]), "loss_last": float(np.mean(log[-20:])),
                              "pilot_s": t_pil, "pilot_vrf": pil["vrf"], "n_paths": N_cv,
                              "run_s": t_run, "total_s": t_pil + t_run,
                              "total_incl_train_s": t_train + t_pil + t_run,
                              "price": run["price"], "std_err": run["std_err"],
                              "vrf": run["vrf"], "plain_price_same_paths": run["plain_price"],
                              "kernel_ms": run["kernel_ms"]}
    out["speedup_excl_train"] = out["plain_fp32"]["total_s"] / out["learned_cv_bf16"]["total_s"]
    out["speedup_incl_train"] = (out["plain_fp32"]["total_s"]
                                 / out["learned_cv_bf16"]["total_incl_train_s"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-1bp", action="store_true")
    ap.add_argument("--hedge-every", type=int, default=8)
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

    c = synth.ASIAN_BARRIER
    N, n = c["n_paths"], c["n_steps"]
    model = mc.Model(kind=mc.MC_GBM, S0=c["S0"], r=c["r"], T=c["T"], sigma=c["sigma"])
    ctx = mc.mc_create(0)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # The control-variate coefficient comes from a pilot on stream tag 1,
    # once, before timing (it is an input of the estimator, not of the step).
    pilot = mc.mc_price(ctx, model, mc.Payoff(mc.MC_ASIAN_ARITH_CALL, c["K"],
                                              cv=mc.MC_CV_GEO_ASIAN), N, n, synth.SEED,
                        mc.Options(pilot_paths=1 << 20))
    beta = pilot["cv_beta"]
    payoffs = [mc.Payoff(mc.MC_ASIAN_ARITH_CALL, c["K"], cv=mc.MC_CV_GEO_ASIAN),
               mc.Payoff(mc.MC_UO_BARRIER_CALL, c["K"], B=c["B"]),
               mc.Payoff(mc.MC_ASIAN_GEO_CALL, c["K"])]
    opts = mc.Options(cv_beta=beta)
    step = mc.PreparedPriceMulti(ctx, model, payoffs, N, n, synth.SEED, opts)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        kernel_ms.append(step()[0].kernel_ms)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = step.results()
    ms = (t1 - t0) * 1e3 / args.steps
    path_steps = N * n
    k_ms = sum(kernel_ms) / len(kernel_ms)
    achieved = SLOTS_PER_PATH_STEP * path_steps / (k_ms * 1e-3)
    line = {
        "metric": "path-steps/s",
        "value": path_steps / (ms * 1e-3),
        "unit": "path-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "GBM arithmetic-Asian (geometric CV) + up-and-out barrier "
                               "(B=130) + geometric Asian on the same paths, 2^24 paths x "
                               "252 log-Euler steps, FP32 state, FP64 reduction, Philox4x32-10",
                   "n_paths": N, "n_steps": n},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_SLOTS / 1e12,
                     "unit": "Tslot/s", "frac": achieved / ALU_PEAK_SLOTS, "traffic": None,
                     "slots_per_path_step": SLOTS_PER_PATH_STEP,
                     "kernel": "gbm_path_kernel<float, asian|geo|uo, log-Euler>"},
        "kernel_ms": k_ms,
        "prices": {"asian_cv": res[0]["price"], "asian_cv_se": res[0]["std_err"],
                   "asian_plain": res[0]["plain_price"], "asian_plain_se": res[0]["plain_std_err"],
                   "uo": res[1]["price"], "uo_se": res[1]["std_err"],
                   "geo": res[2]["price"], "geo_se": res[2]["std_err"], "cv_beta": beta,
                   "vrf": res[0]["vrf"]},
    }
    if not args.no_time_to_1bp:
        line["time_to_1bp"] = time_to_1bp(ctx, mc, synth, hedge_every=args.hedge_every)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
