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
issue peak (it reads and writes no HBM per step); `cpu_baseline` times the
FP64 oracle on a bounded sample of the same workload on the host cores.
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

# MI355X: 256 CUs at 2.4 GHz; one wave64 VALU instruction per clock per CU
# at full rate (4 SIMDs x 16 lanes), i.e. 64 lane-operations per clock per CU.
N_CU, CLOCK_HZ, LANES_PER_CLK = 256, 2.4e9, 64
ALU_PEAK_OPS = N_CU * CLOCK_HZ * LANES_PER_CLK        # 3.93e13 lane-op slots/s

# Issue cost, in full-rate slots, of the instruction classes the method
# needs on gfx950 (measured by paper_1906_02818_amd/isa_rates.hip).
COST_MUL64 = 4.0     # 32x32->64-bit product (v_mad_u64_u32)
COST_TRANS = 4.0     # v_exp/log/sin/cos/sqrt_f32

# Algorithmic operations per path-step of this workload (one normal per step):
#   Philox4x32-10: 10 rounds x (2 mul64 + 2 xor3) per 4 normals
#   uniform: 3 ops per uniform, one uniform per normal
#   Box-Muller: (log, sqrt, sin, cos) + 3 mul per 2 normals
#   step: 1 fma; Asian: exp2 + add; geometric: add; barrier: compare + and
OPS_MUL64 = 5.0
OPS_TRANS = 2.0 + 1.0
OPS_SIMPLE = 5.0 + 3.0 + 1.5 + 1.0 + 1.0 + 1.0 + 2.0
SLOTS_PER_PATH_STEP = OPS_MUL64 * COST_MUL64 + OPS_TRANS * COST_TRANS + OPS_SIMPLE


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    for _ in range(args.warmup):
        mc.mc_price_multi(ctx, model, payoffs, N, n, synth.SEED, opts)
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = mc.mc_price_multi(ctx, model, payoffs, N, n, synth.SEED, opts)
        kernel_ms.append(res[0]["kernel_ms"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
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
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_OPS / 1e12,
                     "unit": "Tslot/s", "frac": achieved / ALU_PEAK_OPS, "traffic": None},
        "kernel_ms": k_ms,
        "prices": {"asian_cv": res[0]["price"], "asian_cv_se": res[0]["std_err"],
                   "asian_plain": res[0]["plain_price"], "asian_plain_se": res[0]["plain_std_err"],
                   "uo": res[1]["price"], "uo_se": res[1]["std_err"],
                   "geo": res[2]["price"], "geo_se": res[2]["std_err"], "cv_beta": beta,
                   "vrf": res[0]["vrf"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
