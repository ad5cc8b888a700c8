"""Regression features and payoffs of the Longstaff-Schwartz tests, written
out in numpy from their definition: monomials of y = S/K of total degree up
to `degree`, by degree and then by the nondecreasing index tuple, followed
by f/K for the max-call on two or more assets."""
import numpy as np

MAXC, PUT, CALL = 1, 2, 3


def payoff(kind, y):
    """f/K per row of y (rows = paths, columns = assets)."""
    if kind == MAXC:
        return np.maximum(y.max(1) - 1.0, 0.0)
    m = y.mean(1)
    return np.maximum(1.0 - m, 0.0) if kind == PUT else np.maximum(m - 1.0, 0.0)


def features(y, f, degree, kind):
    d = y.shape[1]
    cols = [np.ones(len(y))]
    if degree >= 1:
        cols += [y[:, a] for a in range(d)]
    if degree >= 2:
        cols += [y[:, a] * y[:, b] for a in range(d) for b in range(a, d)]
    if degree >= 3:
        cols += [y[:, a] * y[:, b] * y[:, c] for a in range(d) for b in range(a, d)
                 for c in range(b, d)]
    if kind == MAXC and d >= 2:
        cols.append(f)
    return np.stack(cols, 1)
