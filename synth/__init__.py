"""Seeded synthetic workloads for the online functional-connectivity hot path.

This module only draws input signals.  It holds none of the connectivity
arithmetic (no taper, no DFT, no cross-spectra, no metric): the HIP path and
the FP64 oracle both consume what it returns, and share nothing else.

The recordings the paper evaluates on (a simulated two-label MEG scenario at
600 Hz and the MIND median-nerve data set, 265 sources at 1792 Hz; Sec. 2.6)
are not available, so these generators stand in for them with the shapes the
workloads have: sensor-space (306 channels, 1/f background plus coupled
narrow-band sources), source-space (thousands of nodes driven by coupled AR(2)
generators through a sparse mixing), and a serving mix of many sessions.

Every generator returns float64 trials shaped [K][N][M] (trials, nodes,
samples) together with a plain-dict session configuration whose keys mirror
the C configuration struct of the library (n_nodes, n_samples, window_trials,
n_fft, fs_hz, f_lo_hz, f_hi_hz, taper, dpss_nw, dpss_k, metrics, elem).
"""
from __future__ import annotations

import numpy as np

# metric mask bits (same values as the C header)
COH, IMCOH, PLV, PLI, WPLI, USPLI, DSWPLI, COR = 1, 2, 4, 8, 16, 32, 64, 128
ALL8 = 255
XCOR = 256   # cross-correlation (not part of ALL8 nor of the random serving subsets)
SPECTRAL7 = 127
METRIC_NAMES = ["coh", "imcoh", "plv", "pli", "wpli", "uspli", "dswpli", "cor"]
METRIC_BITS = dict(zip(METRIC_NAMES, [COH, IMCOH, PLV, PLI, WPLI, USPLI, DSWPLI, COR]))


def base_config(**kw) -> dict:
    cfg = dict(n_nodes=0, n_samples=0, window_trials=0, n_fft=0, fs_hz=1000.0,
               f_lo_hz=0.0, f_hi_hz=0.0, taper="hann", dpss_nw=0.0, dpss_k=0,
               metrics=ALL8, gram="fp32", elem="f32")
    cfg.update(kw)
    return cfg


# --------------------------------------------------------------------------
# building blocks (signal models only)
# --------------------------------------------------------------------------

def ar2_coeffs(f_hz: np.ndarray, r: np.ndarray, fs: float):
    """Coefficients of a resonant AR(2) with poles r*exp(+-i 2 pi f/fs)."""
    a1 = 2.0 * r * np.cos(2.0 * np.pi * f_hz / fs)
    a2 = -r * r
    return a1, a2


def coupled_ar2(rng, n_gen: int, n_trials: int, n_samp: int, fs: float,
                f_range=(8.0, 30.0), r_range=(0.90, 0.99), density=0.05,
                lag_ms=(5, 40), gain=0.5, burn=300) -> np.ndarray:
    """n_gen resonant AR(2) generators with directed, delayed coupling.

    Edges only run from a lower to a higher generator index (a DAG), so the
    coupled system is stable whenever each AR(2) is.  Each edge e: s -> t
    adds g_e * y_s(n - lag_e) to the innovation of t.  Trials are independent
    realisations (simulated together along a batch axis) after `burn` samples.
    Returns [n_trials][n_gen][n_samp].
    """
    f = rng.uniform(*f_range, size=n_gen)
    r = rng.uniform(*r_range, size=n_gen)
    a1, a2 = ar2_coeffs(f, r, fs)
    src, dst = np.nonzero(np.triu(rng.random((n_gen, n_gen)) < density, k=1))
    lags = rng.integers(int(round(lag_ms[0] * fs / 1000)), int(round(lag_ms[1] * fs / 1000)) + 1,
                        size=src.size)
    g = gain * (1.0 - r[dst]) * rng.choice([-1.0, 1.0], size=src.size)
    max_lag = int(lags.max()) if lags.size else 1
    T = burn + n_samp
    y = np.zeros((T + max_lag + 2, n_trials, n_gen))
    e = rng.standard_normal((T, n_trials, n_gen))
    off = max_lag + 2
    for n in range(T):
        t = n + off
        v = a1 * y[t - 1] + a2 * y[t - 2] + e[n]
        if src.size:
            np.add.at(v, (slice(None), dst), g * y[t - lags, :, src].T)
        y[t] = v
    out = y[off + burn: off + T]                 # [n_samp][n_trials][n_gen]
    return np.ascontiguousarray(out.transpose(1, 2, 0))


def sparse_mixing(rng, n_nodes: int, n_src: int, nnz_per_row: int) -> np.ndarray:
    """Dense matrix holding a sparse leadfield-like mixing: nnz Gaussian
    weights per row at random source columns."""
    L = np.zeros((n_nodes, n_src))
    k = min(nnz_per_row, n_src)
    for i in range(n_nodes):
        cols = rng.choice(n_src, size=k, replace=False)
        L[i, cols] = rng.standard_normal(k)
    return L


def pink_noise(rng, shape_prefix, n_samp: int) -> np.ndarray:
    """Unit-variance 1/f noise: white -> rfft -> scale by f^-1/2 (DC=0) -> irfft."""
    w = rng.standard_normal(tuple(shape_prefix) + (n_samp,))
    W = np.fft.rfft(w, axis=-1)
    f = np.arange(W.shape[-1], dtype=np.float64)
    scale = np.zeros_like(f)
    scale[1:] = 1.0 / np.sqrt(f[1:])
    p = np.fft.irfft(W * scale, n=n_samp, axis=-1)
    p /= p.std(axis=-1, keepdims=True) + 1e-300
    return p


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def c1_tiny(seed: int = 1, n_trials: int = 20):
    """32 nodes, 20 trials x 256 samples at 1 kHz, Hann, 256-point FFT, all
    129 bins, float64 throughout.  10 Hz sinusoids with per-node phase
    offsets ~U(0, 2pi) plus N(0,1) noise, mixed by a 32x32 Gaussian matrix."""
    rng = np.random.default_rng(seed)
    N, M, fs = 32, 256, 1000.0
    phi = rng.uniform(0.0, 2.0 * np.pi, size=N)
    A = rng.standard_normal((N, N))
    t = np.arange(M) / fs
    x = np.empty((n_trials, N, M))
    for k in range(n_trials):
        s = np.sin(2.0 * np.pi * 10.0 * t[None, :] + phi[:, None]) + rng.standard_normal((N, M))
        x[k] = A @ s
    cfg = base_config(n_nodes=N, n_samples=M, window_trials=n_trials, n_fft=256, fs_hz=fs,
                      f_lo_hz=0.0, f_hi_hz=500.0, taper="hann",
                      metrics=COH | PLV | PLI | WPLI, elem="f64")
    return x, cfg


def c2_sensor(seed: int = 2, n_trials: int = 300):
    """306 sensors, 600-sample trials at 1 kHz, 1024-point FFT, 8-30 Hz,
    sliding window of 100 trials, all 8 metrics.  Unit-variance 1/f noise plus
    8 narrow-band 20 Hz AR(2) sources forming 4 driver->follower pairs with
    lags ~U{5..40} ms, spread by a Gaussian 306x8 leadfield at 1:1
    signal:noise power."""
    rng = np.random.default_rng(seed)
    N, M, fs, S = 306, 600, 1000.0, 8
    a1, a2 = ar2_coeffs(np.full(S, 20.0), np.full(S, 0.98), fs)
    lags = rng.integers(5, 41, size=S // 2)
    burn, max_lag = 300, 41
    T = burn + M + max_lag
    e = rng.standard_normal((n_trials, S, T))
    y = np.zeros((n_trials, S, T))
    for n in range(2, T):
        y[:, :, n] = a1 * y[:, :, n - 1] + a2 * y[:, :, n - 2] + e[:, :, n]
    src = np.empty((n_trials, S, M))
    for p in range(S // 2):
        d, f = 2 * p, 2 * p + 1
        st = burn + max_lag
        src[:, d] = y[:, d, st:st + M]
        # follower: the driver delayed by lag_p, plus a weaker own rhythm
        src[:, f] = 0.8 * y[:, d, st - lags[p]:st - lags[p] + M] + 0.6 * y[:, f, st:st + M]
    lead = rng.standard_normal((N, S))
    sig = np.einsum("ns,ksm->knm", lead, src)
    sig /= np.sqrt(np.mean(sig ** 2))
    noise = pink_noise(rng, (n_trials, N), M)
    x = sig + noise
    cfg = base_config(n_nodes=N, n_samples=M, window_trials=100, n_fft=1024, fs_hz=fs,
                      f_lo_hz=8.0, f_hi_hz=30.0, taper="hann", metrics=ALL8, elem="f32")
    return x, cfg


def source_space(seed: int, n_nodes: int, n_trials: int, n_samp: int, n_gen: int,
                 fs: float = 1000.0, nnz_per_row: int = 10, density: float = 0.05,
                 lag_ms=(5, 40)):
    """Source-space activity: coupled AR(2) generators (f ~U(8,30) Hz,
    r ~U(0.90,0.99)) spread by a sparse leadfield-like mixing (nnz Gaussian
    weights per row), plus white noise at the mean signal power."""
    rng = np.random.default_rng(seed)
    g = coupled_ar2(rng, n_gen, n_trials, n_samp, fs, density=density, lag_ms=lag_ms)
    g /= g.std() + 1e-300
    L = sparse_mixing(rng, n_nodes, n_gen, nnz_per_row)
    sig = np.matmul(L[None, :, :], g)                 # [K][N][M]
    p = float(np.mean(sig ** 2))
    x = sig + np.sqrt(p) * rng.standard_normal(sig.shape)
    return x


def c3_source(seed: int = 3, n_trials: int = 50, n_nodes: int = 5000):
    """5000 nodes, 50 trials x 500 samples at 1 kHz, 512-point FFT, 8-30 Hz
    (12 bins), 200 coupled AR(2) generators at 5% directed density with lags
    ~U{5..40} ms, sparse mixing with 10 nonzeros per row, white noise."""
    x = source_space(seed, n_nodes, n_trials, 500, 200)
    cfg = base_config(n_nodes=n_nodes, n_samples=500, window_trials=50, n_fft=512,
                      fs_hz=1000.0, f_lo_hz=8.0, f_hi_hz=30.0, taper="hann",
                      metrics=ALL8, elem="f32")
    return x, cfg


def c4_sessions(seed: int = 4, n_sessions: int = 64):
    """Serving mix: per session N ~ {60,128,306,1000,2000}, W ~ U{10..100},
    each metric bit ~ Bernoulli(1/2) (non-empty), 500-sample trials at 1 kHz,
    512-point FFT, 8-30 Hz.  Returns a list of session configs and the seed
    of each session's trial stream (drawn with `c4_trials`)."""
    rng = np.random.default_rng(seed)
    Ns = np.array([60, 128, 306, 1000, 2000])
    out = []
    for s in range(n_sessions):
        n = int(rng.choice(Ns))
        w = int(rng.integers(10, 101))
        mask = 0
        while mask == 0:
            mask = int(sum(b for b in METRIC_BITS.values() if rng.random() < 0.5))
        cfg = base_config(n_nodes=n, n_samples=500, window_trials=w, n_fft=512,
                          fs_hz=1000.0, f_lo_hz=8.0, f_hi_hz=30.0, taper="hann",
                          metrics=mask, elem="f32")
        out.append((cfg, int(rng.integers(1 << 31))))
    return out


def c4_trials(cfg: dict, stream_seed: int, n_trials: int):
    """Trials for one serving session (C3-style generator, max(10, N/25)
    generators)."""
    n = cfg["n_nodes"]
    return source_space(stream_seed, n, n_trials, cfg["n_samples"], max(10, n // 25))


def c4_arrivals(rng, n_sessions: int, duration_s: float, rate_hz: float = 10.0):
    """Poisson arrivals (exponential gaps, mean 1/rate) per session, merged and
    sorted: returns (times, session index)."""
    ts, ss = [], []
    for s in range(n_sessions):
        t = rng.exponential(1.0 / rate_hz)
        while t < duration_s:
            ts.append(t)
            ss.append(s)
            t += rng.exponential(1.0 / rate_hz)
    order = np.argsort(ts, kind="stable")
    return np.asarray(ts)[order], np.asarray(ss)[order]


def c5_config(**kw):
    cfg = base_config(n_nodes=10000, n_samples=1000, window_trials=200, n_fft=1000,
                      fs_hz=1000.0, f_lo_hz=4.0, f_hi_hz=40.0, taper="dpss",
                      dpss_nw=2.0, dpss_k=3, metrics=ALL8, gram="bf16x3", elem="f32")
    cfg.update(kw)
    return cfg


def c5_multitaper(seed: int = 5, n_trials: int = 200, n_nodes: int = 10000, n_gen: int = 250):
    """Large multitaper workload: n_gen coupled AR(2) generators at 20% directed
    density with lags ~U{1..50} ms spread to n_nodes by a sparse mixing
    (4 nonzeros per row) plus white noise; DPSS NW=2, 3 tapers, 4-40 Hz,
    sliding window of 200 trials of 1000 samples.  Returns float32 trials
    (the size makes float64 pointless: both sides consume float32 input)."""
    rng = np.random.default_rng(seed)
    g = coupled_ar2(rng, n_gen, n_trials, 1000, 1000.0, f_range=(4.0, 40.0),
                    density=0.20, lag_ms=(1, 50), gain=0.25)
    g /= g.std() + 1e-300
    L = sparse_mixing(rng, n_nodes, n_gen, 4).astype(np.float32)
    x = np.empty((n_trials, n_nodes, 1000), dtype=np.float32)
    for k in range(n_trials):
        s = L @ g[k].astype(np.float32)
        p = float(np.mean(s.astype(np.float64) ** 2))
        x[k] = s + np.float32(np.sqrt(p)) * rng.standard_normal((n_nodes, 1000), dtype=np.float32)
    return x, c5_config()


def two_sinusoids(n_trials: int, M: int, F: int, fs: float, f0: float, tau_s: float,
                  seed: int = 0, random_phase: bool = True):
    """Two nodes: x = cos(2 pi f0 t + th_k), y = cos(2 pi f0 (t - tau) + th_k)."""
    rng = np.random.default_rng(seed)
    t = np.arange(M) / fs
    th = rng.uniform(0, 2 * np.pi, size=n_trials) if random_phase else np.full(n_trials, 0.3)
    x = np.empty((n_trials, 2, M))
    x[:, 0] = np.cos(2 * np.pi * f0 * t[None, :] + th[:, None])
    x[:, 1] = np.cos(2 * np.pi * f0 * (t[None, :] - tau_s) + th[:, None])
    return x


def rank1_zero_lag(n_trials: int, N: int, M: int, seed: int = 0):
    """x_i = a_i * s with a_i = +-2^e_i: a single source seen at zero lag, with
    power-of-two gains so every node's spectrum is an exact multiple."""
    rng = np.random.default_rng(seed)
    e = rng.integers(-3, 4, size=N)
    sgn = rng.choice([-1.0, 1.0], size=N)
    a = sgn * np.ldexp(1.0, e)
    s = rng.standard_normal((n_trials, 1, M))
    return a[None, :, None] * s


def zero_lag_mixture(n_trials: int, N: int, M: int, n_src: int = 4, noise: float = 0.5, seed: int = 0):
    """Independent white sources mixed instantaneously (zero lag) plus
    independent sensor noise: no true lagged coupling anywhere."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, n_src))
    s = rng.standard_normal((n_trials, n_src, M))
    return np.matmul(A[None], s) + noise * rng.standard_normal((n_trials, N, M))
