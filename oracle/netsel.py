"""Network post-processing oracle (test infrastructure only, like the rest of
`oracle/`): what the online display path does with a band-mean network.

The paper normalises every network by its maximum edge weight and draws only
the strongest edges (5% of them for the offline figures, 10% in the online
session), with node size given by degree in the thresholded network (results
sections on the simulated and the measured data, and the online pipeline).
Written here as the plain definition over a packed upper-triangle network
w[P], P = N(N-1)/2, pair (i, j), i < j, at i(2N-i-1)/2 + j-i-1:

  finite edges  E = { e : w_e finite }      (USPLI / DSWPLI are NaN for K < 2)
  m             = max_{e in E} |w_e|
  w_norm_e      = w_e / m   (float32 division; 0 when m = 0; non-finite kept)
  k             = min(ceil(f * P), |E|)     f = top fraction in [0, 1]
  T             = k-th largest |w_e| over E (float32), +inf when k = 0
  selected_e    = e in E and |w_e| >= T     (every edge tied with T is kept)
  degree_i      = number of selected edges at node i
  strength_i    = sum of |w_norm_e| over the selected edges at node i (FP64)

Readings: "strongest" and the maximum are taken on |w| so that the signed
ImCoh network keeps its strongest negative edges; ties at the threshold are
all kept, which makes the selected set unique.
"""
from __future__ import annotations

import math

import numpy as np


def pair_endpoints(N: int):
    """(i, j) of every packed index, in packed order."""
    iu = np.triu_indices(N, 1)
    return iu[0].astype(np.int64), iu[1].astype(np.int64)


def network_select(w: np.ndarray, N: int, fraction: float):
    """Returns dict(max_abs, threshold, k, n_finite, n_selected, w_norm,
    selected, degree, strength) for a float32 network w[P]."""
    w = np.asarray(w, dtype=np.float32)
    P = N * (N - 1) // 2
    assert w.shape == (P,)
    fin = np.isfinite(w)
    a = np.abs(w)
    n_fin = int(fin.sum())
    m = np.float32(a[fin].max()) if n_fin else np.float32(0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        if m > 0:
            w_norm = (w / m).astype(np.float32)
        else:
            w_norm = np.where(fin, np.float32(0.0), w).astype(np.float32)
    k = min(int(math.ceil(float(fraction) * P)), n_fin)
    if k > 0:
        T = np.float32(np.sort(a[fin])[::-1][k - 1])
        sel = fin & (a >= T)
    else:
        T = np.float32(np.inf)
        sel = np.zeros(P, dtype=bool)
    pi, pj = pair_endpoints(N)
    degree = np.bincount(pi[sel], minlength=N) + np.bincount(pj[sel], minlength=N)
    s = np.abs(w_norm[sel]).astype(np.float64)
    strength = np.bincount(pi[sel], weights=s, minlength=N) + np.bincount(pj[sel], weights=s, minlength=N)
    return dict(max_abs=float(m), threshold=float(T), k=k, n_finite=n_fin, n_selected=int(sel.sum()),
                w_norm=w_norm, selected=sel, degree=degree.astype(np.int64), strength=strength)
