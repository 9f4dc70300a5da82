"""Time-resolved analytic-signal connectivity on the device (fcx_hilbert_*)
against the oracle (oracle/hilbert.py): the analytic signal element by
element, and every window's seven metrics for every pair (sizes that span
several tiles with a ragged tail, every transform length, windows of one
sample, overlapping windows on both the one-pass block path and the
window-by-window path), plus sampled pairs at 5000 nodes, a zero-lag rank-1
segment (exact zeros) and sinusoids at constant phase offsets.

Tolerances.  The analytic signal: 1e-5 of its largest magnitude, and per node
within the rounding model below.  The metrics: 1e-5 absolute, plus for PLI /
USPLI the oracle's tie allowances, and for WPLI / DSWPLI an allowance
computed on the oracle side alone: the device's z of node i may deviate by
e_i = 2^-22 s_i (s_i = the oracle's tie scale ||x_i||_2 2 log2 F / sqrt F,
about 2^-24 times the FP32 error growth of the transforms, with a margin of
4), so every Im(z_i conj z_j) may move by e_i |z_j| + e_j |z_i|, and with E
the window's sum of those moves (the oracle's tie-threshold sum / 16),
  |d WPLI|   <= 2E / (A - E)                       (full range if A <= E)
  |d DSWPLI| <= 2D / (A^2 - Q - D), D = 4AE + 2E^2  (full range if not > 0)
from the oracle's A = sum |Im| and Q = sum Im^2.  The allowance is capped at
the metric's range, and the share of (pair, window) entries that need it
(error above the base bound) must stay under WIDE_SHARE (it is logged).
Windows whose |Im| sum is within the tie thresholds' sum are degenerate:
WPLI and DSWPLI are ratios of rounding there and may take any value in their
ranges (the same rule as for the trial-based paths); they are left out of
the share."""
import numpy as np
import pytest

import oracle
from gpu_helpers import TOL, log, tie_bounds
from oracle import hilbert as oh
from oracle import stream as so

pytestmark = pytest.mark.gpu

M7 = oracle.METRICS7
BOUND = {"fp32": dict.fromkeys(M7, TOL),
         "bf16x3": dict.fromkeys(M7, TOL),
         "bf16": dict(coh=3e-3, imcoh=TOL, plv=3e-3, pli=TOL, wpli=TOL, uspli=TOL, dswpli=TOL)}


@pytest.fixture(scope="module")
def fcx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2303_03279_amd as m
    return m


def _segment(seed, N, M, fs=1000.0):
    """Nodes that share three sinusoidal sources at node-specific lags, under
    independent white noise of about the same in-band power (float32)."""
    rng = np.random.default_rng(seed)
    t = np.arange(M + 64) / fs
    src = 0.2 * np.stack([np.sin(2 * np.pi * f * t + rng.uniform(0, 2 * np.pi)) for f in (10.0, 17.0, 23.0)])
    x = rng.standard_normal((N, M)).astype(np.float64)
    for i in range(N):
        lag = int(rng.integers(0, 64))
        x[i] += rng.standard_normal(3) @ src[:, lag:lag + M]
    return x.astype(np.float32)


def _taps(T, fs=1000.0, f1=8.0, f2=30.0):
    return np.ones(1) if T == 1 else so.fir_design(so.BANDPASS, fs, f1, f2, n_taps=T)


def _run(fcx, x, taps, L, H, gram="fp32", want_z=True):
    import torch
    N, M = x.shape
    h = fcx.Hilbert(N, M, taps, L, H, gram=gram)
    xd = torch.from_numpy(x).cuda()
    out = torch.full((h.n_windows, 7, h.P), float("nan"), dtype=torch.float32, device="cuda")
    z = torch.empty((M, N, 2), dtype=torch.float32, device="cuda") if want_z else None
    fcx.check(h.run(xd.data_ptr(), M, out.data_ptr(), z.data_ptr() if want_z else 0), "hilbert_run")
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    zc = None
    if want_z:
        zz = z.cpu().numpy()
        zc = (zz[..., 0] + 1j * zz[..., 1]).T.astype(np.complex128)     # [N][M]
    nw, F = h.n_windows, h.fft_len
    fcx.check(h.close())
    return res, zc, nw, F


Z_MODEL = 2.0 ** -22      # device z deviation per node, in units of the node's tie scale
WIDE_SHARE = 0.01         # largest share of (pair, window) entries whose WPLI/DSWPLI error may exceed the base bound


def _check_z_model(z, zr, scale):
    """Every node's analytic signal within the rounding model of the allowance."""
    dev = np.max(np.abs(z - zr), axis=1)
    ratio = dev / np.maximum(scale, 1e-300)
    assert np.all(dev <= Z_MODEL * scale), f"z deviation {float(ratio.max()):.3e} of the tie scale > {Z_MODEL:.3e}"
    return float(ratio.max())


def _rounding_allowance(r):
    """First-order WPLI / DSWPLI bounds from the oracle's window sums (see the
    module docstring), and the degenerate windows (|Im| sum within the tie
    thresholds' sum: any value in the metric's range is correct there)."""
    A, Q, tsum = r["A"][:, 0], r["Q"][:, 0], r["tsum"][:, 0]
    E = tsum * (Z_MODEL / oracle.DELTA_F32)
    D = 4 * A * E + 2 * E * E
    with np.errstate(divide="ignore", invalid="ignore"):
        wpli = np.where(A > E, np.minimum(1.0, 2 * E / (A - E)), 1.0)
        den = A * A - Q - D
        dsw = np.where(den > 0, np.minimum(2.0, 2 * D / den), 2.0)
    deg = A <= tsum
    wpli[deg], dsw[deg] = 1.0, 2.0
    return {"wpli": wpli, "dswpli": dsw}, deg


def _compare(res, ref_windows, bound, label):
    worst, wide, n = {}, {}, 0
    for w, r in enumerate(ref_windows):
        K = r["K"]
        dpli, dus = tie_bounds(r, K)
        cond, deg = _rounding_allowance(r)
        n += int(np.sum(~deg))
        for q, m in enumerate(M7):
            got = res[w, q].astype(np.float64)
            want = r["band"][m]
            if m in ("uspli", "dswpli") and K < 2:
                assert np.all(np.isnan(got)), (label, w, m)
                continue
            err = np.abs(got - want)
            allow = np.full(err.shape, bound[m]) + (dpli if m == "pli" else 0.0) + (dus if m == "uspli" else 0.0)
            allow = allow + cond.get(m, 0.0)
            bad = err > allow
            assert not bad.any(), (f"{label} window {w} {m}: {int(bad.sum())} pairs over, worst {err.max():.3e} "
                                   f"(gpu {got[np.argmax(err)]:.9f}, oracle {want[np.argmax(err)]:.9f})")
            worst[m] = max(worst.get(m, 0.0), float(err.max()) if err.size else 0.0)
            if m in cond:   # entries outside the degenerate windows that need the allowance
                wide[m] = wide.get(m, 0) + int(np.sum((err > bound[m]) & ~deg))
    share = {m: v / max(n, 1) for m, v in wide.items()}
    log(f"{label}: max abs err " + ", ".join(f"{m}={v:.2e}" for m, v in worst.items()) +
        "; share of (pair, window) entries that need the rounding allowance (error above the base bound): " +
        ", ".join(f"{m}={v:.4f}" for m, v in share.items()))
    for m, v in share.items():
        assert v <= WIDE_SHARE or n == 0, (label, m, v)


@pytest.mark.parametrize("N,M,T,L,H", [
    (7, 300, 101, 0, 0),          # F=512, odd N, one window
    (70, 500, 251, 100, 50),      # F=1024, two tile rows with a ragged tail, overlapping windows
    (130, 256, 1, 64, 64),        # F=256, no filter, three tile rows
    (5, 40, 1, 1, 1),             # windows of one sample: USPLI / DSWPLI undefined
    (33, 1500, 301, 700, 500),    # F=2048, a tail of samples after the last window
    (9, 1000, 3001, 250, 250),    # F=4096, a long filter
    (40, 600, 101, 150, 50),      # one pass over blocks of 50 samples, three windows open at a time
    (20, 300, 51, 30, 20),        # blocks of 10 samples (gcd of 30 and 20), windows of 3 blocks every 2
    (20, 200, 51, 10, 4),         # blocks of 2 samples: window by window
])
def test_analytic_and_windows_vs_oracle(fcx, N, M, T, L, H):
    x = _segment(N * 7 + M, N, M)
    taps = _taps(T)
    log(f"hilbert N={N} M={M} T={T} L={L} H={H}")
    res, z, nw, F = _run(fcx, x, taps, L, H)
    assert F == oh.fft_len(M, T)
    zr = oh.analytic(x.astype(np.float64), taps)
    zerr = np.max(np.abs(z - zr)) / np.max(np.abs(zr))
    sc = oh.tie_scale(x, F)
    zm = _check_z_model(z, zr, sc)
    log(f"  F={F} windows={nw}: analytic max rel err {zerr:.2e}, per-node deviation {zm:.2e} of the tie scale")
    assert zerr <= TOL
    ref = oh.network(zr, L, H, scale=sc)
    assert nw == len(ref)
    _compare(res, ref, BOUND["fp32"], f"N={N} M={M} T={T}")


@pytest.mark.parametrize("gram", ["bf16x3", "bf16"])
def test_gram_precisions(fcx, gram):
    N, M, T, L, H = 96, 400, 151, 200, 100
    x = _segment(5, N, M)
    taps = _taps(T)
    res, z, _, F = _run(fcx, x, taps, L, H, gram=gram)
    zr = oh.analytic(x.astype(np.float64), taps)
    sc = oh.tie_scale(x, F)
    _check_z_model(z, zr, sc)
    ref = oh.network(zr, L, H, scale=sc)
    _compare(res, ref, BOUND[gram], f"gram {gram}")


def test_metric_subset_leaves_other_rows(fcx):
    import torch
    N, M = 40, 200
    x = _segment(9, N, M)
    taps = _taps(51)
    h = fcx.Hilbert(N, M, taps, 100, 100, metrics=fcx.FCX_PLV | fcx.FCX_WPLI)
    xd = torch.from_numpy(x).cuda()
    out = torch.full((h.n_windows, 7, h.P), 7.0, dtype=torch.float32, device="cuda")
    fcx.check(h.run(xd.data_ptr(), M, out.data_ptr()))
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    fcx.check(h.close())
    assert np.all(res[:, [0, 1, 3, 5, 6]] == 7.0)
    ref = oh.network(oh.analytic(x.astype(np.float64), taps), 100, 100)
    for w, r in enumerate(ref):
        assert np.max(np.abs(res[w, 2] - r["band"]["plv"])) <= TOL
        assert np.max(np.abs(res[w, 4] - r["band"]["wpli"])) <= TOL


def test_full_size_sampled_pairs(fcx):
    """5000 nodes, 500 samples at 1 kHz, an 8-12 Hz band-pass with a 4 Hz
    transition (825 taps, F=2048), windows of 100 samples every 50: sampled
    rows x sampled columns against the oracle, and a repeat run bitwise
    equal."""
    import torch
    N, M, fs = 5000, 500, 1000.0
    rng = np.random.default_rng(77)
    x = _segment(77, N, M)
    taps = so.fir_design(so.BANDPASS, fs, 8.0, 12.0, transition_hz=4.0)
    assert taps.size == 825
    log(f"hilbert full size N={N} M={M} T={taps.size}")
    h = fcx.Hilbert(N, M, taps, 100, 50)
    xd = torch.from_numpy(x).cuda()
    out = torch.empty((h.n_windows, 7, h.P), dtype=torch.float32, device="cuda")
    zd = torch.empty((M, N, 2), dtype=torch.float32, device="cuda")
    fcx.check(h.run(xd.data_ptr(), M, out.data_ptr(), zd.data_ptr()))
    torch.cuda.synchronize()
    rows = np.sort(rng.choice(N - 1, 24, replace=False))
    cols = np.sort(rng.choice(N, 160, replace=False))
    cols = np.unique(np.concatenate([cols, [N - 1, N - 2]]))
    pi, pj = [], []
    for r in rows:
        for c in cols:
            if c > r:
                pi.append(r)
                pj.append(c)
    pi, pj = np.array(pi), np.array(pj)
    nodes = np.unique(np.concatenate([pi, pj]))
    loc = {int(n): k for k, n in enumerate(nodes)}
    zr = oh.analytic(x[nodes].astype(np.float64), taps)
    ref = oh.network(zr, 100, 50, pi=[loc[int(a)] for a in pi], pj=[loc[int(b)] for b in pj],
                     scale=oh.tie_scale(x[nodes], h.fft_len))
    idx = oracle.packed_index(pi, pj, N)
    res = out[:, :, torch.from_numpy(idx).cuda()].cpu().numpy()
    assert h.n_windows == len(ref) == 9
    la = np.array([loc[int(a)] for a in pi])
    lb = np.array([loc[int(b)] for b in pj])
    zs = zd[:, torch.from_numpy(nodes).cuda()].cpu().numpy()
    zdev = (zs[..., 0] + 1j * zs[..., 1]).T.astype(np.complex128)
    e = float(np.max(np.abs(zdev - zr)))
    zm = _check_z_model(zdev, zr, oh.tie_scale(x[nodes], h.fft_len))
    log(f"  analytic max rel err {e / np.max(np.abs(zr)):.2e} on the sampled nodes, "
        f"per-node deviation {zm:.2e} of the tie scale")
    assert e <= TOL * np.max(np.abs(zr))
    _compare(res, ref, BOUND["fp32"], f"N={N} sampled {pi.size} pairs")
    out2 = torch.empty_like(out)
    fcx.check(h.run(xd.data_ptr(), M, out2.data_ptr()))
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    fcx.check(h.close())


def test_smallest_segment(fcx):
    """Two nodes and one sample: one window of one sample (PLV = PLI = WPLI =
    COH = 1 for non-zero samples, USPLI / DSWPLI undefined)."""
    x = np.array([[0.7], [-1.3]], dtype=np.float32)
    taps = np.ones(1)
    res, z, nw, F = _run(fcx, x, taps, 0, 0)
    assert nw == 1 and F == 256 and res.shape == (1, 7, 1)
    zr = oh.analytic(x.astype(np.float64), taps)
    assert np.max(np.abs(z - zr)) <= TOL * np.max(np.abs(zr))
    ref = oh.network(zr, scale=oh.tie_scale(x, F))
    _compare(res, ref, BOUND["fp32"], "N=2 M=1")


def test_nonfinite_sample_poisons_its_transform_pair_only(fcx):
    """A NaN in node 5 makes the analytic signals of nodes 4 and 5 (one
    transform) non-finite, so the metrics of the pairs touching them are
    meaningless; every other pair equals the run on clean data bit for bit."""
    N, M = 12, 300
    x = _segment(21, N, M)
    taps = _taps(101)
    clean, _, _, _ = _run(fcx, x, taps, 100, 100, want_z=False)
    x2 = x.copy()
    x2[5, 17] = np.nan
    dirty, _, _, _ = _run(fcx, x2, taps, 100, 100, want_z=False)
    pi, pj = oracle.all_pairs(N)
    hit = np.isin(pi, [4, 5]) | np.isin(pj, [4, 5])
    assert np.array_equal(dirty[:, :, ~hit], clean[:, :, ~hit])
    assert not np.array_equal(dirty[:, :, hit], clean[:, :, hit], equal_nan=True)


@pytest.mark.parametrize("L,H", [(100, 100), (100, 50)])
def test_rank1_zero_lag_exact(fcx, L, H):
    """One source seen at zero lag with power-of-two gains.  Nodes 2m and
    2m + 1 share one transform (x_2m + i x_2m+1), and the gains scale node
    pairs (2m, 2m + 1) together (x_2m = c_m x_0, x_2m+1 = c_m x_1 with
    x_1 = d x_0), so every transform is an exact multiple of the first and
    z_i = c z_j holds bit for bit between nodes of the same parity: for those
    pairs IMCOH = PLI = WPLI = DSWPLI = 0 exactly and USPLI = -1/(K-1).  Pairs
    of mixed parity come out of one transform's real and imaginary halves,
    whose rounding differs; they are compared with the oracle under the tie
    and rounding allowances like every other pair.  Windows that do not
    overlap run the batch pair pass per window, overlapping ones the one-pass
    block kernel."""
    N, M, T = 24, 400, 101
    rng = np.random.default_rng(12)
    s0 = rng.standard_normal(M)
    c = np.ldexp(1.0, rng.integers(-3, 4, size=N // 2)) * rng.choice([-1.0, 1.0], size=N // 2)
    x = np.empty((N, M))
    x[0::2] = c[:, None] * s0[None, :]
    x[1::2] = -0.5 * c[:, None] * s0[None, :]
    x = x.astype(np.float32)
    taps = _taps(T)
    res, z, nw, F = _run(fcx, x, taps, L, H)
    pi, pj = oracle.all_pairs(N)
    same = (pi % 2) == (pj % 2)
    for w in range(nw):
        for q, m in enumerate(M7):
            if m in ("imcoh", "pli", "wpli", "dswpli"):
                assert np.all(res[w, q, same] == 0.0), (w, m, float(np.max(np.abs(res[w, q, same]))))
        us = res[w, M7.index("uspli"), same].astype(np.float64)
        assert np.max(np.abs(us + 1.0 / (L - 1))) <= 1e-6
    zr = oh.analytic(x.astype(np.float64), taps)
    sc = oh.tie_scale(x, F)
    _check_z_model(z, zr, sc)
    _compare(res, oh.network(zr, L, H, scale=sc), BOUND["fp32"], "rank-1 zero lag")


@pytest.mark.parametrize("gram", ["fp32", "bf16"])
def test_constant_phase_offsets(fcx, gram):
    """Sinusoids of one frequency at node-specific phase offsets, no noise:
    inside a window every z_i conj z_j keeps its phase, so PLV = PLI = WPLI =
    USPLI = DSWPLI = COH = 1 and IMCOH = sin of the offset, away from the
    filter's edge transients (the oracle gives the values with them); the
    device against the oracle, and the windows clear of the segment's edges
    against the closed forms."""
    N, M, T, fs, f0 = 10, 1200, 201, 1000.0, 20.0
    rng = np.random.default_rng(31)
    ph = rng.uniform(0.3, 2.8, size=N) * np.where(np.arange(N) % 3 == 0, -1.0, 1.0)
    t = np.arange(M) / fs
    x = np.cos(2 * np.pi * f0 * t[None, :] + ph[:, None]).astype(np.float32)
    taps = so.fir_design(so.BANDPASS, fs, 10.0, 30.0, n_taps=T)
    L, H = 200, 200
    res, z, nw, F = _run(fcx, x, taps, L, H, gram=gram)
    zr = oh.analytic(x.astype(np.float64), taps)
    sc = oh.tie_scale(x, F)
    ref = oh.network(zr, L, H, scale=sc)
    _compare(res, ref, BOUND[gram], f"constant phase offsets {gram}")
    pi, pj = oracle.all_pairs(N)
    d = ph[pi] - ph[pj]
    for w in range(2, nw - 2):          # clear of the edge transients
        for m in ("coh", "plv", "pli", "wpli", "uspli", "dswpli"):
            got = res[w, M7.index(m)].astype(np.float64)
            assert np.max(np.abs(got - 1.0)) <= 1e-3 + BOUND[gram][m], (w, m)
        imc = res[w, M7.index("imcoh")].astype(np.float64)
        assert np.max(np.abs(imc - np.sin(d))) <= 1e-3 + BOUND[gram]["imcoh"], w
