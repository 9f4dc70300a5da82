"""Pins of the network post-processing oracle (oracle/netsel.py) against
things it does not share code with: a pure-Python dense-matrix brute force
on tiny networks, closed forms (a star, all-equal weights, the 0 and 1
fractions) and invariants."""
import math

import numpy as np
import pytest

from oracle import netsel


def _brute(w, N, fraction):
    """Dense N x N symmetric matrix, Python lists and sorted() only."""
    W = [[None] * N for _ in range(N)]
    e = 0
    for i in range(N):
        for j in range(i + 1, N):
            W[i][j] = W[j][i] = float(w[e])
            e += 1
    fin = [(abs(W[i][j]), i, j) for i in range(N) for j in range(i + 1, N) if math.isfinite(W[i][j])]
    m = max((a for a, _, _ in fin), default=0.0)
    P = N * (N - 1) // 2
    k = min(math.ceil(fraction * P), len(fin))
    keys = sorted((a for a, _, _ in fin), reverse=True)
    T = keys[k - 1] if k > 0 else math.inf
    chosen = {(i, j) for a, i, j in fin if k > 0 and a >= T}
    deg = [0] * N
    stren = [0.0] * N
    for (i, j) in chosen:
        v = abs(float(np.float32(np.float32(W[i][j]) / np.float32(m)))) if m > 0 else 0.0
        deg[i] += 1
        deg[j] += 1
        stren[i] += v
        stren[j] += v
    return m, T, k, chosen, deg, stren


@pytest.mark.parametrize("N,fraction,seed", [(7, 0.05, 0), (7, 0.3, 1), (9, 0.5, 2), (12, 0.1, 3), (5, 1.0, 4),
                                             (6, 0.0, 5)])
def test_brute_force(N, fraction, seed):
    rng = np.random.default_rng(seed)
    P = N * (N - 1) // 2
    w = rng.standard_normal(P).astype(np.float32)
    w[rng.integers(P)] = np.nan                   # a non-finite edge is never kept
    r = netsel.network_select(w, N, fraction)
    m, T, k, chosen, deg, stren = _brute(w, N, fraction)
    assert r["max_abs"] == np.float32(m)
    assert r["k"] == k and r["threshold"] == np.float32(T)
    pi, pj = netsel.pair_endpoints(N)
    got = {(int(pi[e]), int(pj[e])) for e in np.flatnonzero(r["selected"])}
    assert got == chosen
    assert list(r["degree"]) == deg
    assert np.allclose(r["strength"], stren, rtol=1e-12, atol=0)


def test_closed_forms():
    N = 10
    P = N * (N - 1) // 2
    pi, pj = netsel.pair_endpoints(N)
    # a star: the 9 strongest edges all touch node 0
    w = np.full(P, 0.1, dtype=np.float32)
    w[pi == 0] = np.linspace(0.5, 0.9, N - 1).astype(np.float32)
    r = netsel.network_select(w, N, 9 / P)
    assert r["k"] == 9 and r["n_selected"] == 9
    assert r["degree"][0] == 9 and all(r["degree"][1:] == 1)
    assert r["max_abs"] == np.float32(0.9) and r["threshold"] == np.float32(0.5)
    assert r["strength"][0] == pytest.approx(float(np.sum(np.abs(w[pi == 0] / np.float32(0.9)))), rel=1e-7)
    # all weights equal: any k >= 1 keeps every edge (ties at the threshold)
    r = netsel.network_select(np.full(P, 0.25, dtype=np.float32), N, 0.01)
    assert r["k"] == 1 and r["n_selected"] == P and all(r["degree"] == N - 1)
    # fraction 1 keeps all finite edges, fraction 0 none
    w = np.random.default_rng(1).uniform(-1, 1, P).astype(np.float32)
    assert netsel.network_select(w, N, 1.0)["n_selected"] == P
    r0 = netsel.network_select(w, N, 0.0)
    assert r0["n_selected"] == 0 and r0["threshold"] == np.inf and all(r0["degree"] == 0)
    # an all-zero network normalises to zeros
    r = netsel.network_select(np.zeros(P, dtype=np.float32), N, 0.5)
    assert r["max_abs"] == 0.0 and not np.any(r["w_norm"])


def test_invariants_and_signed_edges():
    rng = np.random.default_rng(7)
    N = 40
    P = N * (N - 1) // 2
    w = rng.uniform(-1, 0.3, P).astype(np.float32)   # strongest edges are negative (ImCoh-like)
    r = netsel.network_select(w, N, 0.05)
    sel = r["selected"]
    assert r["n_selected"] == r["k"] == math.ceil(0.05 * P)   # distinct weights: exactly k
    assert np.all(w[sel] < 0)
    assert r["degree"].sum() == 2 * r["n_selected"]
    assert r["strength"].sum() == pytest.approx(2 * np.abs(r["w_norm"][sel].astype(np.float64)).sum(), rel=1e-12)
    fin = np.isfinite(r["w_norm"])
    assert np.max(np.abs(r["w_norm"][fin])) == 1.0
    assert np.all(np.abs(w[sel]) >= np.max(np.abs(w[~sel])))
