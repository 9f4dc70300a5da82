"""Shared helpers of the GPU parity tests: run a session through the C ABI
and compare its networks with the FP64 oracle, element by element."""
from __future__ import annotations

import sys

import numpy as np

import oracle

TOL = 1e-5          # FP32 path: absolute error on the [-1, 1] metric scale
TOL_F64 = 1e-11     # FP64 path


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def run_pushes(fcx, cfg, x, start=0, stop=None, session=None):
    """Push trials x[start:stop] (host path) and return the session."""
    s = session or fcx.Session(cfg)
    dt = np.float64 if cfg.get("elem", "f32") == "f64" else np.float32
    stop = x.shape[0] if stop is None else stop
    for k in range(start, stop):
        fcx.check(s.push_host(np.ascontiguousarray(x[k], dtype=dt)), f"push {k}")
    return s


def tie_bounds(ref, K):
    """Per-pair band-mean allowances for PLI and USPLI from the oracle's tie
    counts: a tie may flip its sign (|G| moves by at most 2 per tie)."""
    G = np.abs(ref["G"]).astype(np.float64)
    t = ref["ties"].astype(np.float64)
    B = G.shape[1]
    dpli = (2 * t / K).sum(axis=1) / B
    if K >= 2:
        dus = (K / (K - 1.0) * (4 * t * G + 4 * t * t) / (K * K)).sum(axis=1) / B
    else:
        dus = np.zeros(G.shape[0])
    return dpli, dus


def degenerate_bounds(ref):
    """Per-pair band-mean allowances for WPLI and DSWPLI from the oracle's
    sums: in a bin whose |Im| sum A is within the sum of the trials' tie
    thresholds, every cross-spectrum's imaginary part may be rounding alone,
    so WPLI = |sum Im| / A and DSWPLI are ratios of rounding and any value in
    their ranges ([0, 1] and [-1, 1]) is correct there."""
    deg = (ref["A"] <= ref["tsum"]).astype(np.float64)
    B = deg.shape[1]
    return deg.sum(axis=1) / B, 2.0 * deg.sum(axis=1) / B


def allowances(ref, K):
    """Extra allowance per metric and pair on top of the base tolerance."""
    dpli, dus = tie_bounds(ref, K)
    dw, dds = degenerate_bounds(ref)
    return {"pli": dpli, "uspli": dus, "wpli": dw, "dswpli": dds}


def compare_network(s, ref, cfg, metrics, idx=None, tol=TOL, label=""):
    """Compare band-mean networks of session s with oracle result ref.
    idx: packed indices of the oracle's pairs (default: all pairs in order)."""
    K = ref["K"]
    extra = allowances(ref, K)
    worst = {}
    for m in metrics:
        st, out, k = s.read(m)
        assert k == K, (m, k, K)
        got = out.astype(np.float64)
        if idx is not None:
            got = got[idx]
        want = ref["band"][m]
        if m in ("uspli", "dswpli") and K < 2:
            assert np.all(np.isnan(got)), m
            continue
        err = np.abs(got - want)
        allow = np.full(err.shape, tol) + extra.get(m, 0.0)
        bad = err > allow
        worst[m] = float(err.max()) if err.size else 0.0
        assert not bad.any(), (
            f"{label} {m}: {int(bad.sum())} pairs over tolerance, worst {err.max():.3e} "
            f"at {int(np.argmax(err))} (gpu {got[np.argmax(err)]:.9f}, oracle {want[np.argmax(err)]:.9f})")
    log(f"{label} K={K} max abs err per metric: " + ", ".join(f"{m}={v:.2e}" for m, v in worst.items()))
    return worst
