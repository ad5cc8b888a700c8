"""Pins of the oracle's Sobol' generator and randomised QMC basket (Sec. IV-B,
Sec. VI-D): the primitive-polynomial list against brute force and the count
formula phi(2^s - 1)/s, dimension 0 against the van der Corput sequence,
the (0, m, 1)-net property of every dimension and the (0, m, 2)-net property
of dimensions (0, 1), the integration error of a smooth product function,
and the randomised estimator of the geometric basket against its closed
form, with an RMSE that falls faster than Monte Carlo's N^(-1/2)."""
import math

import numpy as np
import pytest

import oracle
import synth
from closed_forms import geo_basket_call

SEED = synth.SEED


def euler_phi(n):
    out, m, q = n, n, 2
    while q * q <= m:
        if m % q == 0:
            while m % q == 0:
                m //= q
            out -= out // q
        q += 1
    if m > 1:
        out -= out // m
    return out


def order_of_x(p, s):
    # Multiplicative order of x modulo p by direct iteration.
    r, k = 2, 1
    while True:
        if r == 1:
            return k
        r <<= 1
        if r >> s & 1:
            r ^= p
        k += 1
        if k > (1 << s):
            return None


def test_primitive_polynomials_brute_force():
    deg, poly = oracle.sobol_polys(200)
    # complete, ordered list for degrees up to 9, by brute force
    brute = []
    for s in range(1, 10):
        for c in range((1 << s) | 1, 2 << s, 2):
            if order_of_x(c, s) == (1 << s) - 1 or (s == 1 and c == 3):
                brute.append((s, c))
    got = [(int(a), int(b)) for a, b in zip(deg, poly) if a <= 9]
    assert got == brute
    for s in range(1, 10):
        assert sum(1 for a in deg if a == s) == euler_phi((1 << s) - 1) // s


def test_dimension_zero_is_van_der_corput():
    V = oracle.sobol_dirs(1)
    P = oracle.sobol_points(V, 1024)[:, 0]
    for i in range(1024):
        rev = int(format(i, "032b")[::-1], 2)
        assert P[i] == rev


@pytest.mark.parametrize("m", [1, 3, 6, 10])
def test_every_dimension_is_a_0m1_net(m):
    V = oracle.sobol_dirs(40)
    P = oracle.sobol_points(V, 1 << m)
    for j in range(40):
        top = np.sort(P[:, j] >> (32 - m))
        assert np.array_equal(top, np.arange(1 << m)), j


def test_first_two_dimensions_are_a_0m2_net():
    m = 8
    V = oracle.sobol_dirs(2)
    P = oracle.sobol_points(V, 1 << m)
    for k in range(m + 1):
        a = P[:, 0] >> (32 - k) if k else np.zeros(1 << m, np.uint32)
        b = P[:, 1] >> (32 - (m - k)) if m - k else np.zeros(1 << m, np.uint32)
        cells = set(zip(a.tolist(), b.tolist()))
        assert len(cells) == 1 << m, k


def test_smooth_integrand_error_is_quasi_monte_carlo():
    # prod_j (1 + (x_j - 1/2)) integrates to 1 on [0,1]^8. At 2^14 Sobol'
    # points the error is a small fraction of the Monte Carlo standard error,
    # and it falls by far more than the Monte Carlo factor 4 from 2^10.
    err = {}
    for n in (1 << 10, 1 << 14):
        P = (oracle.sobol_points(oracle.sobol_dirs(8), n).astype(np.float64) + 0.5) / 2.0 ** 32
        f = np.prod(1.0 + (P - 0.5), axis=1)
        err[n] = (abs(f.mean() - 1.0), f.std() / math.sqrt(n))
    e14, se14 = err[1 << 14]
    assert e14 < 0.1 * se14
    assert err[1 << 10][0] / e14 > 6.0


def test_rqmc_geometric_basket_closed_form_and_rate():
    d = 16
    sigma, corr, _ = synth.basket_market(d)
    L = oracle.cholesky(corr)
    S0 = np.full(d, 100.0)
    w = np.full(d, 1.0 / d)
    exact = geo_basket_call(S0, sigma, corr, w, 0.05, 1.0, 100.0)
    R = 16
    rmse = []
    Ns = [1 << 8, 1 << 10, 1 << 12]
    for N in Ns:
        est = [oracle.basket_qmc(S0, sigma, L, w, 0.05, 1.0, 100.0, 1, N, SEED, r)[:, 1].mean()
               for r in range(R)]
        est = np.array(est)
        rmse.append(math.sqrt(np.mean((est - exact) ** 2)))
        if N == Ns[-1]:
            se = est.std(ddof=1) / math.sqrt(R)
            assert abs(est.mean() - exact) < 4 * se
    slope = np.polyfit(np.log(Ns), np.log(rmse), 1)[0]
    assert slope < -0.7, (slope, rmse)
