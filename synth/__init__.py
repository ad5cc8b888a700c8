"""Seeded synthetic inputs shared by the tests, the oracle runs and the bench.

This module holds NO arithmetic of the Monte Carlo method: it only states the
workload parameters and draws the synthetic market data (per-asset
volatilities and the correlation matrix of the basket) from numpy's seeded
generator. The random numbers the method itself draws (the path normals) are
not made here: each side generates them from Philox4x32-10 on its own.
"""
from __future__ import annotations

import numpy as np

SEED = 1234

# European call on 1-D GBM (the paper's vanilla-call experiment, Sec. VI-A.1,
# at the money): log-Euler, 64 steps, 2^18 paths, double precision.
EURO = dict(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, n_steps=64,
            n_paths=1 << 18)

# The paper's own vanilla-call instance (strike 120), Sec. VI-A.1.
PAPER_VANILLA = dict(S0=100.0, K=120.0, r=0.05, sigma=0.2, T=1.0)

# Arithmetic Asian call and discretely monitored up-and-out call on one set of
# GBM paths: 252 steps, 2^24 paths, single-precision path state.
ASIAN_BARRIER = dict(S0=100.0, K=100.0, B=130.0, r=0.03, sigma=0.25, T=1.0,
                     n_steps=252, n_paths=1 << 24)

# Heston arithmetic Asian call, full-truncation Euler, 256 steps, 2^22 paths.
HESTON = dict(S0=100.0, v0=0.04, kappa=2.0, theta=0.04, xi=0.5, rho=-0.7,
              r=0.02, T=1.0, K=100.0, n_steps=256, n_paths=1 << 22)

# Learned control variate on the Heston Asian: 2000 Adam steps on a fixed
# 2^20-path training set (minibatch 2^15), evaluated on 2^24 fresh paths.
# Adam: lr 3.2e-2, dropped by 4x every 800 steps (moments kept), beta2 0.95.
# Chosen by the variance reduction on 2^22 fresh paths: with beta2 0.999,
# Adam's second moment remembers the large gradients of the first steps for
# ~1000 steps and the steps shrink (2000 steps at a constant 4e-3: VRF
# 12.86); with beta2 0.95 the dropped rate reaches 13.50 at minibatch 2^16
# (13.47 with another training seed; lr 1.6e-2: 13.47; drops every 700
# steps: 13.48; 1000 steps with drops every 400: 13.43). Minibatch 2^15
# reaches 13.47 (lr 2.2e-2: 13.46; 1.6e-2: 13.44; another training seed:
# 13.43) in two thirds of the time; 2^14 reaches 13.43 and is barely faster,
# the step time being then set by the kernels' latency, not their work.
LEARNED_CV = dict(n_train=1 << 20, batch=1 << 15, adam_steps=2000, lr=3.2e-2, beta2=0.95,
                  decay=0.25, decay_every=800, n_eval=1 << 24)

# Basket call on d = 256 correlated GBM assets, 100 steps, 2^20 paths.
BASKET = dict(d=256, S0=100.0, K=100.0, r=0.05, T=1.0, n_steps=100,
              n_paths=1 << 20)


def basket_market(d: int = 256, seed: int = SEED):
    """Synthetic stand-in for the paper's historical covariance (Sec. VI-A.2,
    Russell 3000 data, not available): per-asset volatilities uniform in
    [0.1, 0.4] and a correlation C = D^{-1/2} (0.3 11^T + 0.7 I + 0.1 G G^T/d)
    D^{-1/2} with G standard normal, D the diagonal of the bracket.

    Returns (sigma[d], corr[d, d], min eigenvalue of corr).
    """
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((d, d))
    sigma = 0.1 + 0.3 * rng.random(d)
    M = 0.3 * np.ones((d, d)) + 0.7 * np.eye(d) + 0.1 * (G @ G.T) / d
    s = 1.0 / np.sqrt(np.diag(M))
    corr = M * s[:, None] * s[None, :]
    corr = 0.5 * (corr + corr.T)
    np.fill_diagonal(corr, 1.0)
    lam_min = float(np.linalg.eigvalsh(corr)[0])
    return sigma, corr, lam_min


def glorot_mlp(seed: int = SEED) -> np.ndarray:
    """Initial weights of the 4-64-64-1 hedge network: Glorot-uniform
    matrices, zero biases, flat layout W1[64][4], b1, W2[64][64], b2, W3[64], b3."""
    rng = np.random.default_rng(seed + 4)

    def glorot(fan_out, fan_in):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, (fan_out, fan_in))

    parts = [glorot(64, 4).ravel(), np.zeros(64), glorot(64, 64).ravel(),
             np.zeros(64), glorot(1, 64).ravel(), np.zeros(1)]
    theta = np.concatenate(parts)
    assert theta.size == 4545
    return theta
