"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a
pure-Python brute force written from the definitions, numpy/scipy library
routines, closed forms, exact special cases, null statistics and invariants.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import brute

M7 = oracle.METRICS7


def _cfg(M, F, fs=1000.0, f_lo=0.0, f_hi=None, taper="hann", nw=0.0, k=0, elem="f64"):
    return synth.base_config(n_nodes=0, n_samples=M, window_trials=0, n_fft=F, fs_hz=fs,
                             f_lo_hz=f_lo, f_hi_hz=fs / 2 if f_hi is None else f_hi,
                             taper=taper, dpss_nw=nw, dpss_k=k, elem=elem)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("F", [16, 32])
@pytest.mark.parametrize("taper", ["hann", "dpss"])
def test_brute_force_tiny(F, taper):
    """Every metric, every bin (DC..Nyquist), all pairs of a tiny random case
    agree with the pure-Python definitions to 1e-12."""
    rng = np.random.default_rng(11 + F)
    K, N, M = 5, 4, 16
    x = rng.standard_normal((K, N, M))
    cfg = _cfg(M, F, taper=taper, nw=1.5, k=2)
    res = oracle.network(x, cfg, with_cor=True)
    tap, lam = oracle.taper_of(cfg)
    bins = list(range(F // 2 + 1))
    assert list(res["bins"]) == bins
    xl = x.tolist()
    for p, (i, j) in enumerate(zip(res["pi"], res["pj"])):
        ref = brute.pair_metrics(xl, int(i), int(j), tap.tolist(), lam.tolist(), bins, F)
        for b, r in enumerate(ref):
            for m in M7:
                assert res["per_bin"][m][p, b] == pytest.approx(r[m], abs=1e-12), (m, i, j, b)
            assert res["G"][p, b] == r["G"]
            if not r["any_zero_sign"]:
                # Vinck's pairwise form equals the closed form when no sign is 0
                assert r["uspli_pairwise"] == pytest.approx(r["uspli"], abs=1e-12)
        for m in M7:
            band = np.mean([r[m] for r in ref])
            assert res["band"][m][p] == pytest.approx(band, abs=1e-12)
        assert res["band"]["cor"][p] == pytest.approx(brute.cor(xl, int(i), int(j)), abs=1e-12)


# ------------------------------------------------------------ library routines

def test_spectra_match_rfft():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, 6, 600))
    cfg = _cfg(600, 1024, f_lo=8, f_hi=30)
    X, l1, lam, bins = oracle.spectra(x, cfg)
    w = oracle.hann_periodic(600)
    ref = np.fft.rfft(w[None, None, :] * x, n=1024, axis=-1)[:, :, bins]
    assert np.max(np.abs(X[:, :, 0, :] - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.allclose(l1[:, :, 0], np.sum(np.abs(w * x), axis=-1), rtol=1e-14)


def test_hann_closed_form():
    w = oracle.hann_periodic(8)
    assert np.allclose(w, [0, 0.1464466094, 0.5, 0.8535533906, 1, 0.8535533906, 0.5, 0.1464466094])


@pytest.mark.parametrize("M,NW,K", [(1000, 2.0, 3), (64, 1.5, 2), (255, 3.0, 5)])
def test_dpss_matches_scipy(M, NW, K):
    from scipy.signal.windows import dpss as sp_dpss
    tap, lam = oracle.dpss(M, NW, K)
    ref, ratios = sp_dpss(M, NW, K, return_ratios=True)
    assert np.allclose(np.sum(tap ** 2, axis=1), 1.0, atol=1e-12)
    for k in range(K):
        assert np.allclose(tap[k], ref[k], atol=1e-9), k
    assert np.allclose(lam, ratios, atol=1e-9)
    assert np.all(np.diff(lam) < 0) and lam[0] < 1.0


def test_cor_matches_corrcoef():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((7, 5, 50))
    x[:, 1] += 0.8 * x[:, 0]
    pi, pj = oracle.all_pairs(5)
    c = oracle.cor(x, pi, pj)
    ref = np.mean([np.corrcoef(x[k])[pi, pj] for k in range(7)], axis=0)
    assert np.allclose(c, ref, atol=1e-13)


# ------------------------------------------------------------------ band plan

@pytest.mark.parametrize("F,fs,lo,hi,nb,first", [
    (512, 1000.0, 8, 30, 12, 4),     # source-space workload: 12 bins
    (1000, 1000.0, 4, 40, 37, 4),    # large multitaper workload: 37 bins
    (1024, 1000.0, 4, 40, 37, 4),    # same count with a 1024-point FFT
    (1024, 1000.0, 8, 30, 23, 8),    # sensor-space workload
    (256, 1000.0, 0, 500, 129, 0),   # tiny workload: all one-sided bins
])
def test_band_plan(F, fs, lo, hi, nb, first):
    b = oracle.band_bins(F, fs, lo, hi)
    assert b.size == nb and b[0] == first


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("tau_ms", [5.0, 12.0, 31.0])
def test_two_sinusoids_constant_lag(tau_ms):
    """x = cos(w t + th_k), y = cos(w (t - tau) + th_k), f0 on a bin, F = M,
    periodic Hann: every trial has CSD proportional to exp(i w tau), so
    COH = PLV = PLI = WPLI = USPLI = DSWPLI = 1 and IMCOH = sin(w tau)."""
    M = F = 200
    fs, f0 = 1000.0, 20.0          # 20 Hz is bin 4 at 5 Hz resolution
    x = synth.two_sinusoids(30, M, F, fs, f0, tau_ms / 1000.0, seed=3)
    cfg = _cfg(M, F, f_lo=f0, f_hi=f0)
    r = oracle.network(x, cfg)
    assert list(r["bins"]) == [4]
    for m in ["coh", "plv", "pli", "wpli", "uspli", "dswpli"]:
        assert r["band"][m][0] == pytest.approx(1.0, abs=1e-12), m
    assert r["band"]["imcoh"][0] == pytest.approx(math.sin(2 * math.pi * f0 * tau_ms / 1000.0), abs=1e-12)


def test_two_sinusoids_constant_phase_any_padding():
    """With the same phase in every trial the CSD repeats exactly, so the
    phase metrics are 1 at every bin with a non-zero imaginary part, for any
    taper and padding; COH is 1 for a single taper (with several tapers the
    taper-combined CSD obeys only Cauchy-Schwarz, COH <= 1)."""
    x = synth.two_sinusoids(12, 150, 256, 1000.0, 23.3, 0.007, seed=1, random_phase=False)
    for taper in ["hann", "dpss"]:
        cfg = _cfg(150, 256, f_lo=10, f_hi=40, taper=taper, nw=2.0, k=3)
        r = oracle.network(x, cfg)
        if taper == "hann":
            assert np.allclose(r["per_bin"]["coh"], 1.0, atol=1e-12)
        else:
            assert np.all(r["per_bin"]["coh"] <= 1.0 + 1e-12)
        assert np.allclose(r["per_bin"]["plv"], 1.0, atol=1e-12)
        assert np.allclose(r["per_bin"]["pli"], 1.0, atol=1e-12)
        assert np.allclose(r["per_bin"]["wpli"], 1.0, atol=1e-12)
        assert np.allclose(r["per_bin"]["uspli"], 1.0, atol=1e-12)
        assert np.allclose(r["per_bin"]["dswpli"], 1.0, atol=1e-12)


def test_rank1_zero_lag_exact():
    """A single source seen with power-of-two gains: every cross-spectrum is
    real, so IMCOH = PLI = WPLI = DSWPLI = 0 exactly, USPLI = -1/(K-1),
    and COH = PLV = |COR| = 1."""
    K, N, M = 9, 6, 128
    x = synth.rank1_zero_lag(K, N, M, seed=4)
    cfg = _cfg(M, 256, f_lo=0, f_hi=500)
    r = oracle.network(x, cfg)
    for m in ["imcoh", "pli", "wpli", "dswpli"]:
        assert np.all(r["per_bin"][m] == 0.0), m
    assert np.all(r["per_bin"]["uspli"] == -1.0 / (K - 1))
    assert np.allclose(r["per_bin"]["coh"], 1.0, atol=1e-13)
    assert np.allclose(r["per_bin"]["plv"], 1.0, atol=1e-13)
    assert np.allclose(np.abs(r["band"]["cor"]), 1.0, atol=1e-13)


def test_dc_and_nyquist_are_real():
    """At DC and Nyquist every spectrum is real: the sign-based metrics vanish
    and USPLI = -1/(K-1)."""
    rng = np.random.default_rng(2)
    K = 7
    x = rng.standard_normal((K, 5, 256))
    cfg = _cfg(256, 256)
    r = oracle.network(x, cfg)
    for b in (0, 128):
        for m in ["imcoh", "pli", "wpli", "dswpli"]:
            assert np.all(r["per_bin"][m][:, b] == 0.0), (m, b)
        assert np.all(r["per_bin"]["uspli"][:, b] == -1.0 / (K - 1))
        assert np.all(r["ties"][:, b] == K)


def test_tie_count_interior_bin():
    """Tie counts at an interior bin: trials in which node 1 is node 0 at
    zero lag (twice the amplitude, so Im CSD is an exact 0), plus a lagged
    component of relative size eps.  With the FP32 threshold eps = 0 and 1e-9
    give |Im| far below it (ties) and eps = 1e-3 far above it; with the FP64
    threshold only eps = 0 is a tie.  The count must be exactly the number of
    tie trials, every nonzero eps must count in G, and a bin of only zero-lag
    trials has its |Im| sum within the tie-threshold sum (the degenerate-bin
    rule)."""
    M = F = 256
    k0 = 20
    f0 = 1000.0 * k0 / F
    t = np.arange(M) / 1000.0
    eps = [0.0, 1e-9, 1e-3, 0.0, 1e-3, 1e-9, 1e-3]
    rng = np.random.default_rng(5)
    x = np.empty((len(eps), 3, M))
    for k, e in enumerate(eps):
        th = rng.uniform(0, 2 * np.pi)
        s = np.cos(2 * np.pi * f0 * t + th)
        lagged = np.cos(2 * np.pi * f0 * t + th - np.pi / 2)
        x[k, 0] = s
        x[k, 1] = 2.0 * s + e * lagged
        x[k, 2] = -4.0 * s
    for elem, n_tie in (("f32", 4), ("f64", 2)):
        # FP32 spectra: threshold 2^-18 of the scale, so eps = 1e-9 is a tie;
        # FP64: 2^-44, so only the exact zeros are
        cfg = _cfg(M, F, f_lo=f0, f_hi=f0, elem=elem)
        r = oracle.network(x, cfg, pi=[0, 0], pj=[1, 2])
        assert list(r["bins"]) == [k0]
        assert r["ties"][0, 0] == n_tie, elem
        assert r["ties"][1, 0] == len(eps)          # exact multiples: every trial a tie
        assert r["G"][1, 0] == 0 and r["A"][1, 0] == 0.0
        assert r["A"][1, 0] <= r["tsum"][1, 0]      # a degenerate bin
        assert r["A"][0, 0] > r["tsum"][0, 0]       # the lagged trials carry real |Im|
        assert abs(r["G"][0, 0]) == sum(1 for e in eps if e > 0.0)


@pytest.mark.parametrize("taper", ["hann", "dpss"])
def test_incremental_equals_plain(taper):
    """The incremental CPU method (running sums, add the new trial and
    subtract the evicted one) gives the plain window recompute's networks at
    every push, through the fill and many evictions."""
    rng = np.random.default_rng(23)
    T, N, M, W = 14, 6, 64, 5
    x = rng.standard_normal((T, N, M))
    x[:, 1, 2:] += 0.8 * x[:, 0, :-2]
    cfg = _cfg(M, 64, f_lo=50, f_hi=300, taper=taper, nw=1.5, k=2)
    pi, pj = oracle.all_pairs(N)
    sl = oracle.Sliding(cfg, N, pi, pj, W)
    for k in range(T):
        band = sl.push(x[k])
        ref = oracle.network(x[max(0, k + 1 - W):k + 1], cfg, pi, pj, with_cor=False)
        for m in M7:
            if ref["K"] < 2 and m in ("uspli", "dswpli"):
                assert np.all(np.isnan(band[m])), (k, m)
                continue
            assert np.max(np.abs(band[m] - ref["band"][m])) < 1e-11, (k, m)


# ------------------------------------------------------------------ statistics

def test_null_statistics_zero_lag_mixture():
    """Zero-lag mixing of independent sources plus noise has no lagged
    coupling: the debiased estimators (IMCOH, USPLI, DSWPLI) average to 0
    within 4 standard errors while PLI sits at its bias sqrt(2/(pi K)) and the
    plain squared WPLI stays positive."""
    K, N, M = 400, 12, 64
    x = synth.zero_lag_mixture(K, N, M, n_src=4, noise=1.0, seed=8)
    cfg = _cfg(M, 64, f_lo=50, f_hi=450)
    r = oracle.network(x, cfg)
    for m in ["imcoh", "uspli", "dswpli"]:
        v = r["per_bin"][m].ravel()
        assert abs(v.mean()) < 4 * v.std() / math.sqrt(v.size), m
    pli = r["per_bin"]["pli"].ravel()
    assert abs(pli.mean() - math.sqrt(2 / (math.pi * K))) < 0.2 * math.sqrt(2 / (math.pi * K))
    assert np.mean(r["per_bin"]["wpli"] ** 2) > 5 * abs(np.mean(r["per_bin"]["dswpli"]))


def test_lagged_pair_detected():
    """The sensor-space workload's driver->follower sources (lags of 5-40 ms)
    give a lagged pair: its PLI/WPLI stands far above the null level."""
    K, M = 100, 600
    rng = np.random.default_rng(0)
    x = synth.two_sinusoids(K, M, 1024, 1000.0, 20.0, 0.012, seed=5)
    x += 1.0 * rng.standard_normal(x.shape)
    cfg = _cfg(M, 1024, f_lo=18, f_hi=22)
    r = oracle.network(x, cfg)
    assert r["band"]["pli"][0] > 0.6 and r["band"]["wpli"][0] > 0.6
    assert r["band"]["imcoh"][0] > 0.1


# ------------------------------------------------------------------ invariants

def _random_case(seed=21, K=15, N=7, M=96):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, N))
    s = rng.standard_normal((K, N, M))
    # add some lagged structure so the imaginary parts are not symmetric
    s[:, 1, 3:] += 0.7 * s[:, 0, :-3]
    return np.matmul(A[None], s)


def test_ranges():
    x = _random_case()
    K = x.shape[0]
    r = oracle.network(x, _cfg(96, 128, f_lo=0, f_hi=500))
    pb = r["per_bin"]
    for m in ["coh", "plv", "pli", "wpli"]:
        assert np.all(pb[m] >= 0) and np.all(pb[m] <= 1 + 1e-12), m
    assert np.all(np.abs(pb["imcoh"]) <= pb["coh"] + 1e-12)
    assert np.all(pb["dswpli"] <= 1 + 1e-12)
    assert np.all(pb["uspli"] >= -1.0 / (K - 1) - 1e-12)
    assert np.all(np.abs(r["band"]["cor"]) <= 1 + 1e-12)


def test_swap_is_hermitian():
    x = _random_case()
    cfg = _cfg(96, 128, f_lo=0, f_hi=500)
    pi, pj = oracle.all_pairs(7)
    a = oracle.network(x, cfg, pi, pj)
    b = oracle.network(x, cfg, pj, pi)
    for m in M7:
        sgn = -1.0 if m == "imcoh" else 1.0
        assert np.allclose(a["per_bin"][m], sgn * b["per_bin"][m], atol=1e-12), m
    assert np.allclose(a["band"]["cor"], b["band"]["cor"], atol=1e-14)


def test_trial_permutation_invariance():
    x = _random_case()
    cfg = _cfg(96, 128, f_lo=0, f_hi=500)
    perm = np.random.default_rng(1).permutation(x.shape[0])
    a = oracle.network(x, cfg)
    b = oracle.network(x[perm], cfg)
    for m in M7 + ["cor"]:
        assert np.allclose(a["band"][m], b["band"][m], atol=1e-12), m


def test_node_permutation_equivariance():
    x = _random_case()
    N = x.shape[1]
    cfg = _cfg(96, 128, f_lo=0, f_hi=500)
    perm = np.random.default_rng(2).permutation(N)
    inv = np.argsort(perm)
    a = oracle.network(x, cfg)
    b = oracle.network(x[:, perm, :], cfg)
    # pair (i, j) of x is pair (inv[i], inv[j]) of the permuted input
    for p, (i, j) in enumerate(zip(a["pi"], a["pj"])):
        u, v = inv[i], inv[j]
        q = oracle.packed_index(min(u, v), max(u, v), N)
        for m in M7:
            sgn = -1.0 if (m == "imcoh" and u > v) else 1.0
            assert a["band"][m][p] == pytest.approx(sgn * b["band"][m][q], abs=1e-12), m
        assert a["band"]["cor"][p] == pytest.approx(b["band"]["cor"][q], abs=1e-12)


def test_scale_laws():
    x = _random_case()
    cfg = _cfg(96, 128, f_lo=0, f_hi=500)
    a = oracle.network(x, cfg)
    y = x.copy()
    y[:, 0] *= 3.5
    y[:, 2] *= -0.25
    b = oracle.network(y, cfg)
    flip = np.where((a["pi"] == 2) | (a["pj"] == 2), -1.0, 1.0)
    for m in M7:
        f = flip if m == "imcoh" else 1.0
        assert np.allclose(a["band"][m], f * b["band"][m], atol=1e-12), m
    assert np.allclose(a["band"]["cor"], flip * b["band"]["cor"], atol=1e-12)


def test_k_below_two():
    x = _random_case(K=1)
    r = oracle.network(x, _cfg(96, 128, f_lo=0, f_hi=500))
    assert np.all(np.isnan(r["per_bin"]["uspli"])) and np.all(np.isnan(r["per_bin"]["dswpli"]))
    assert np.all((r["per_bin"]["pli"] == 1.0) | (r["per_bin"]["pli"] == 0.0))


def test_debiased_wpli_reading():
    """The debiased squared WPLI is the pairwise (j != k) form; the printed
    'WPLI^2' differs from it and is not the estimator used."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((6, 3, 32))
    cfg = _cfg(32, 32)
    r = oracle.network(x, cfg)
    tap, lam = oracle.taper_of(cfg)
    ref = brute.pair_metrics(x.tolist(), 0, 1, tap.tolist(), lam.tolist(), [5], 32)[0]
    assert r["per_bin"]["dswpli"][0, 5] == pytest.approx(ref["dswpli"], abs=1e-12)
    assert abs(r["per_bin"]["dswpli"][0, 5] - r["per_bin"]["wpli"][0, 5] ** 2) > 1e-3
