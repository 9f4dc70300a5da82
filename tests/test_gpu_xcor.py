"""XCOR on the device (FFT correlation per pair, maximum over the lags, window
sum with a ring of per-trial maxima) against the FP64 oracle's literal
time-domain XCOR over the same window of float32-rounded trials."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, log, run_pushes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fcx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2303_03279_amd as m
    return m


def _check(s, x, cfg, lo, hi, label, pi=None, pj=None, idx=None, tol=TOL):
    N = cfg["n_nodes"]
    if pi is None:
        pi, pj = oracle.all_pairs(N)
    L = cfg.get("xcor_max_lag", 0) or cfg["n_samples"] - 1
    ref = oracle.xcor(oracle.as_device_input(x[lo:hi], cfg), pi, pj, max_lag=L)
    st, got, K = s.read("xcor")
    assert st == 0 and K == hi - lo, (st, K)
    got = got.astype(np.float64)
    if idx is not None:
        got = got[idx]
    err = float(np.max(np.abs(got - ref)))
    log(f"xcor {label}: K={K} L={L} max abs err {err:.2e} (values {ref.min():.3f}..{ref.max():.3f})")
    assert err <= tol, (label, err)


@pytest.mark.parametrize("N,M,W,T,L", [(40, 100, 5, 9, 0), (70, 256, 4, 7, 0), (33, 300, 3, 5, 60),
                                       (65, 500, 6, 11, 0), (20, 600, 3, 4, 0), (17, 1000, 2, 3, 1000 - 1)])
def test_sliding_window_vs_oracle(fcx, N, M, W, T, L):
    """Windows that fill and evict, FFT lengths 256..2048 (every radix set of
    the transform), full and limited lag ranges, ragged tiles."""
    cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=max(M, 256), f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.XCOR | synth.COR | synth.COH, xcor_max_lag=L)
    x = synth.source_space(40 + N, N, T, M, 6).astype(np.float32)
    x[:, 3, 11:] += 0.9 * x[:, 2, :-11]           # a lagged copy: a large XCOR at lag -11
    s = run_pushes(fcx, cfg, x, stop=W - 1)
    _check(s, x, cfg, 0, W - 1, f"N={N} M={M} filling")
    run_pushes(fcx, cfg, x, start=W - 1, session=s)
    _check(s, x, cfg, T - W, T, f"N={N} M={M} W={W} sliding")
    s.close()


def test_xcor_only_session_and_resync(fcx):
    """A session with XCOR alone; resync (replay of the cached window) gives
    the same network bit for bit; one trial in the window."""
    N, M, W = 50, 200, 4
    cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=256, f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.XCOR)
    x = synth.source_space(3, N, 7, M, 5).astype(np.float32)
    s = run_pushes(fcx, cfg, x, stop=1)
    _check(s, x, cfg, 0, 1, "one trial")
    run_pushes(fcx, cfg, x, start=1, session=s)
    a = s.read("xcor")[1].copy()
    fcx.check(s.resync())
    b = s.read("xcor")[1]
    assert np.array_equal(a, b)
    _check(s, x, cfg, 7 - W, 7, "after resync")
    s.close()


def test_degenerate_rows_and_transients(fcx):
    """A constant node (zero energy: XCOR 0 against it) and a node whose
    energy sits in the first samples (tiny overlaps at large lags)."""
    N, M, W = 12, 128, 3
    cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=128, f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.XCOR)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((5, N, M)).astype(np.float32)
    x[:, 0, :] = 3.0
    x[:, 1, 20:] *= 1e-3
    s = run_pushes(fcx, cfg, x)
    _check(s, x, cfg, 5 - W, 5, "constant and transient rows")
    s.close()


@pytest.mark.parametrize("N", [2, 3, 5, 63, 64, 65, 129])
def test_node_counts_and_tile_edges(fcx, N):
    """The smallest networks (one pair; an odd count, so the last column pair
    holds a missing node) and counts at and around the 64-node tile edge,
    with a lagged copy between the first two nodes."""
    M, W, T = 120, 3, 5
    cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=128, f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.XCOR)
    rng = np.random.default_rng(100 + N)
    x = rng.standard_normal((T, N, M)).astype(np.float32)
    x[:, 1, 7:] += 0.8 * x[:, 0, :-7]
    s = run_pushes(fcx, cfg, x)
    _check(s, x, cfg, T - W, T, f"N={N}")
    s.close()


@pytest.mark.parametrize("L", [0, 50])
def test_tail_lags(fcx, L):
    """Lags whose overlap holds under 1/1024 of the advanced node's energy
    (summed directly): white noise (short tails at the last samples), a
    decaying transient (a tail of most lags), and a node of zero-mean
    integers followed by exact zeros (zero suffix energy from sample 80 on,
    so its XCOR there is 0 and its sums stop at sample 80)."""
    N, M, W, T = 10, 200, 3, 4
    cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=256, f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.XCOR, xcor_max_lag=L)
    rng = np.random.default_rng(31 + L)
    x = rng.standard_normal((T, N, M)).astype(np.float32)
    h = rng.integers(-5, 6, size=(T, 80))
    h[:, -1] -= h.sum(axis=1)
    x[:, 4] = 0.0
    x[:, 4, :80] = h
    x[:, 5] *= np.exp(-np.arange(M) / 15.0).astype(np.float32)
    x[:, 6, 9:] += 0.7 * x[:, 5, :-9]
    s = run_pushes(fcx, cfg, x)
    _check(s, x, cfg, T - W, T, f"tails L={L}")
    s.close()


def test_batch_then_read(fcx):
    """After a batch pass the XCOR sums come from the replay of the window."""
    N, M, W = 60, 300, 5
    cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=512, f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.XCOR | synth.COH)
    x = synth.source_space(12, N, W, M, 6).astype(np.float32)
    import torch
    s = fcx.Session(cfg)
    xd = torch.from_numpy(x).cuda()
    torch.cuda.synchronize()
    fcx.check(s.push_batch_device(xd.data_ptr(), W, N * M, M))
    fcx.check(s.sync())
    _check(s, x, cfg, 0, W, "batch")
    s.close()


def test_source_size_sampled_rows(fcx):
    """1000 nodes, 500-sample trials (F = 1024), sampled rows against all
    columns."""
    N, M, W, T = 1000, 500, 3, 4
    cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=512, f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.XCOR)
    x = synth.source_space(5, N, T, M, 40).astype(np.float32)
    s = run_pushes(fcx, cfg, x)
    rows = [0, 1, 499, 998]
    pi, pj = oracle.row_pairs(rows, N)
    _check(s, x, cfg, T - W, T, "N=1000 sampled rows", pi=pi, pj=pj, idx=oracle.packed_index(pi, pj, N))
    s.close()


def test_served_xcor_rejected(fcx):
    srv = fcx.Server(1 << 30)
    cfg = synth.base_config(n_nodes=20, n_samples=100, window_trials=3, n_fft=128, f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.XCOR)
    st, h = srv.open(cfg)
    assert st == fcx.FCX_E_INVAL and h is None
    fcx.check(srv.destroy())


def test_f64_session(fcx):
    """An FP64 session with XCOR and COH: XCOR runs its FP32 transform (FP32
    tolerance), COH stays at the FP64 bound, after the window slides."""
    from gpu_helpers import TOL_F64, compare_network
    N, M, W, T = 40, 200, 3, 5
    cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=256, f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.XCOR | synth.COH)
    cfg["elem"] = "f64"
    x = synth.source_space(17, N, T, M, 5)
    s = run_pushes(fcx, cfg, x)
    _check(s, x, cfg, T - W, T, "f64 session")
    ref = oracle.network(oracle.as_device_input(x[T - W:], cfg), cfg)
    compare_network(s, ref, cfg, ["coh"], tol=TOL_F64, label="f64 session coh")
    s.close()
