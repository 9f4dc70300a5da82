"""Pins of the oracle's XCOR (oracle.xcor / orc_xcor) against what it does not
share code with: the printed formula as pure-Python loops (1-based t), a
numpy.correlate evaluation of the whole lag curve, closed forms (identical
signals and an exactly delayed copy reach 1 at a known lag), the zero-lag
case equal to COR, and invariants (range, symmetry, scale and offset)."""
import math

import numpy as np
import pytest

import oracle


def _xcor_literal(x, y, L):
    """The XCOR equation with t = 1..N as printed, both lag directions,
    maximised; returns (max value, its lag)."""
    M = len(x)
    xb = sum(x) / M
    yb = sum(y) / M

    def one(u, ub, v, vb, tau):
        num = sum((u[t + tau - 1] - ub) * (v[t - 1] - vb) for t in range(1, M - tau + 1))
        eu = sum((u[t + tau - 1] - ub) ** 2 for t in range(1, M - tau + 1))
        ev = sum((v[t - 1] - vb) ** 2 for t in range(1, M + 1))
        d = math.sqrt(eu * ev)
        return num / d if d > 0 else 0.0

    best, lag = -math.inf, 0
    for s in range(-L, L + 1):
        r = one(x, xb, y, yb, s) if s >= 0 else one(y, yb, x, xb, -s)
        if r > best:
            best, lag = r, s
    return best, lag


def _xcor_numpy(x, y, L):
    """Whole lag curve from numpy.correlate and cumulative energies."""
    xt, yt = x - x.mean(), y - y.mean()
    M = len(x)
    full = np.correlate(xt, yt, mode="full")          # index M-1+s: sum_t xt[t+s] yt[t]
    sx = np.cumsum((xt ** 2)[::-1])[::-1]             # sx[tau] = sum_{t>=tau} xt[t]^2
    sy = np.cumsum((yt ** 2)[::-1])[::-1]
    vals = []
    for s in range(-L, L + 1):
        num = full[M - 1 + s]
        d = math.sqrt((sx[s] * sy[0]) if s >= 0 else (sy[-s] * sx[0]))
        vals.append(num / d if d > 0 else 0.0)
    return np.array(vals)


@pytest.mark.parametrize("M,L,seed", [(10, 9, 0), (12, 5, 1), (9, 0, 2), (16, 15, 3)])
def test_literal_formula(M, L, seed):
    rng = np.random.default_rng(seed)
    K, N = 2, 4
    x = rng.standard_normal((K, N, M))
    pi, pj = oracle.all_pairs(N)
    got, lag = oracle.xcor(x, pi, pj, max_lag=L, with_lag=True)
    for p in range(pi.size):
        vals = [_xcor_literal(list(x[k, pi[p]]), list(x[k, pj[p]]), L) for k in range(K)]
        assert got[p] == pytest.approx(sum(v for v, _ in vals) / K, abs=1e-12)
        assert lag[p] == vals[-1][1]


def test_numpy_correlate_curve():
    rng = np.random.default_rng(4)
    K, N, M = 3, 6, 64
    x = rng.standard_normal((K, N, M))
    x[:, 1, 5:] += 0.8 * x[:, 0, :-5]                 # node 1 lags node 0 by 5 samples
    pi, pj = oracle.all_pairs(N)
    for L in (M - 1, 20):
        got = oracle.xcor(x, pi, pj, max_lag=L)
        ref = [np.mean([_xcor_numpy(x[k, a], x[k, b], L).max() for k in range(K)]) for a, b in zip(pi, pj)]
        assert np.allclose(got, ref, atol=1e-12, rtol=0)


def test_closed_forms():
    rng = np.random.default_rng(5)
    M, d = 40, 7
    v = rng.standard_normal(M - d)
    v -= v.mean()
    y = np.concatenate([v, np.zeros(d)])               # zero mean
    x = np.concatenate([np.zeros(d), v])               # x(t + d) = y(t) on the whole support
    z = rng.standard_normal(M)
    trials = np.stack([np.stack([x, y, z, 3.0 * z + 2.0])])
    val, lag = oracle.xcor(trials, [0, 1, 2], [1, 0, 3], with_lag=True)
    assert val[0] == pytest.approx(1.0, abs=1e-14) and lag[0] == d      # x advanced by d matches y
    assert val[1] == pytest.approx(1.0, abs=1e-14) and lag[1] == -d     # same pair, other order
    assert val[2] == pytest.approx(1.0, abs=1e-14) and lag[2] == 0      # affine copy: lag 0


def test_zero_lag_is_cor_and_invariants():
    rng = np.random.default_rng(6)
    K, N, M = 4, 8, 50
    x = rng.standard_normal((K, N, M))
    pi, pj = oracle.all_pairs(N)
    assert np.allclose(oracle.xcor(x, pi, pj, max_lag=0), oracle.cor(x, pi, pj), atol=1e-14, rtol=0)
    full = oracle.xcor(x, pi, pj)
    assert np.all(full <= 1.0 + 1e-12) and np.all(full >= -1.0 - 1e-12)
    assert np.all(full >= oracle.xcor(x, pi, pj, max_lag=0) - 1e-15)   # more lags never lower the max
    assert np.array_equal(full, oracle.xcor(x, pj, pi))                 # symmetric in the pair order
    y = x.copy()
    y[:, 3] = 2.5 * y[:, 3] - 7.0                                       # positive scale and offset
    assert np.allclose(full, oracle.xcor(y, pi, pj), atol=1e-12, rtol=0)
