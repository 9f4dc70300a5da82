"""FP64 CPU oracle for the online all-to-all functional-connectivity path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the HIP path; both only consume the seeded inputs of
`synth`.

What it computes is the plain definition of the metrics (supplementary metric
section, time and frequency domain) recomputed over the trials it is handed:
taper and direct DFT at the band bins (`orc_spectra` in oracle.c), per-trial
CSD/PSD and their trial sums, the seven spectral metrics per bin and their
band mean (`orc_pairs`), and the trial-averaged Pearson correlation
(`orc_cor`).  The taper (periodic Hann, or DPSS by Slepian's tridiagonal
eigenproblem with concentration ratios), and the band plan are defined here.

Pins (tests/test_oracle_pins.py): pure-Python brute force on tiny inputs
(oracle/brute.py), numpy.fft.rfft and numpy.corrcoef, scipy's DPSS, closed
forms for two sinusoids at a constant lag, exact zeros for a rank-1 zero-lag
mixture, DC/Nyquist bins, statistics under the null, and invariants.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

METRICS7 = ["coh", "imcoh", "plv", "pli", "wpli", "uspli", "dswpli"]

# tie factors: FP32 spectra on the device side, FP64 spectra on the device side
DELTA_F32 = 2.0 ** -18
DELTA_F64 = 2.0 ** -44


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64, I32, D = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.orc_spectra.argtypes = [P, I64, I64, I64, I64, P, I32, I64, P, I32, P, I64, P, P, P]
        lib.orc_spectra.restype = None
        lib.orc_pairs.argtypes = [P, P, P, I64, I64, I32, I32, P, P, P, I64, D, P, P, P, P, P, P]
        lib.orc_pairs.restype = None
        lib.orc_slide.argtypes = [P, P, P, P, I32, I64, I32, I32, P, P, P, I64, I64, P, P, P]
        lib.orc_slide.restype = None
        lib.orc_cor.argtypes = [P, I64, I64, I64, I64, P, P, I64, P]
        lib.orc_cor.restype = None
        lib.orc_xcor.argtypes = [P, I64, I64, I64, I64, I64, P, P, I64, P, P]
        lib.orc_xcor.restype = None
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# band plan and tapers
# --------------------------------------------------------------------------

def band_bins(n_fft: int, fs: float, f_lo: float, f_hi: float) -> np.ndarray:
    """Bins k_lo..k_hi inclusive with k = floor(f * F / fs) (clamped to the
    one-sided range); reproduces 12 bins for 8-30 Hz at F=512 and 37 bins for
    4-40 Hz at F=1000."""
    lo = max(0, int(math.floor(f_lo * n_fft / fs + 1e-9)))
    hi = min(n_fft // 2, int(math.floor(f_hi * n_fft / fs + 1e-9)))
    return np.arange(lo, hi + 1, dtype=np.int32)


def hann_periodic(M: int) -> np.ndarray:
    n = np.arange(M, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * n / M)


def dpss(M: int, NW: float, K: int):
    """Discrete prolate spheroidal sequences: the K eigenvectors with the
    largest eigenvalues of Slepian's symmetric tridiagonal matrix
    (diagonal ((M-1)/2 - n)^2 cos(2 pi W), off-diagonal n(M-n)/2, W = NW/M),
    unit energy; even orders have a positive sum, odd orders a positive first
    significant sample.  Concentration ratios are w^T A w with the sinc
    kernel A_mn = sin(2 pi W (m-n)) / (pi (m-n)), A_nn = 2W.
    Returns (tapers [K][M], ratios [K])."""
    from scipy.linalg import eigh_tridiagonal
    W = NW / M
    n = np.arange(M, dtype=np.float64)
    d = ((M - 1 - 2 * n) / 2.0) ** 2 * np.cos(2 * np.pi * W)
    e = n[1:] * (M - n[1:]) / 2.0
    vals, vecs = eigh_tridiagonal(d, e, select="i", select_range=(M - K, M - 1))
    tap = vecs[:, ::-1].T.copy()
    tap /= np.linalg.norm(tap, axis=1, keepdims=True)
    thresh = max(1e-7, 1.0 / M)
    for k in range(K):
        if k % 2 == 0:
            if tap[k].sum() < 0:
                tap[k] *= -1
        else:
            first = tap[k][tap[k] ** 2 > thresh][0]
            if first < 0:
                tap[k] *= -1
    m = n[:, None] - n[None, :]
    with np.errstate(invalid="ignore", divide="ignore"):
        A = np.sin(2 * np.pi * W * m) / (np.pi * m)
    A[np.arange(M), np.arange(M)] = 2 * W
    ratios = np.einsum("km,mn,kn->k", tap, A, tap)
    return tap, ratios


def taper_of(cfg: dict):
    """(tapers [L][M], weights [L]) for a session configuration."""
    M = int(cfg["n_samples"])
    if cfg.get("taper", "hann") == "hann":
        return hann_periodic(M)[None, :], np.ones(1)
    tap, lam = dpss(M, float(cfg["dpss_nw"]), int(cfg["dpss_k"]))
    return tap, lam


def packed_index(i, j, N):
    """Index of pair (i, j), i < j, in the row-major upper triangle without
    the diagonal."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    return i * (2 * N - i - 1) // 2 + (j - i - 1)


def all_pairs(N: int):
    i, j = np.triu_indices(N, k=1)
    return i.astype(np.int64), j.astype(np.int64)


def row_pairs(rows, N: int, cols=None):
    """Pairs (i, j), i < j, for i in rows and j in cols (default: all j > i)."""
    pi, pj = [], []
    for r in rows:
        cs = np.arange(r + 1, N) if cols is None else np.asarray([c for c in cols if c > r])
        pi.append(np.full(cs.size, r, dtype=np.int64))
        pj.append(cs.astype(np.int64))
    return np.concatenate(pi), np.concatenate(pj)


# --------------------------------------------------------------------------
# the oracle
# --------------------------------------------------------------------------

def spectra(x: np.ndarray, cfg: dict, nodes=None):
    """Complex spectra [K][nn][L][B] and per-taper L1 norms [K][nn][L]."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    K, N, M = x.shape
    tap, lam = taper_of(cfg)
    tap = np.ascontiguousarray(tap, dtype=np.float64)
    L = tap.shape[0]
    bins = band_bins(int(cfg["n_fft"]), float(cfg["fs_hz"]), float(cfg["f_lo_hz"]), float(cfg["f_hi_hz"]))
    B = bins.size
    nodes = np.arange(N, dtype=np.int32) if nodes is None else np.ascontiguousarray(nodes, dtype=np.int32)
    nn = nodes.size
    Xre = np.empty((K, nn, L, B))
    Xim = np.empty((K, nn, L, B))
    l1 = np.empty((K, nn, L))
    lib.orc_spectra(_ptr(x), K, N * M, M, M, _ptr(tap), L, int(cfg["n_fft"]), _ptr(bins), B,
                    _ptr(nodes), nn, _ptr(Xre), _ptr(Xim), _ptr(l1))
    return Xre + 1j * Xim, l1, lam, bins


def network(x: np.ndarray, cfg: dict, pi=None, pj=None, delta=None, with_sums=False,
            with_cor=True) -> dict:
    """Metrics over all trials of x ([K][N][M], float64) for pairs (pi, pj)
    (default: every pair i < j in packed order).

    Returns a dict with band means `band[m]` ([np]), per-bin values
    `per_bin[m]` ([np][B]), sign sums `G` and tie counts `ties` ([np][B]),
    the |Im| and Im^2 sums `A`, `Q` and the sum of the trials' tie thresholds
    `tsum` ([np][B]), `cor` ([np]) and `K`.
    """
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    K, N, M = x.shape
    if pi is None:
        pi, pj = all_pairs(N)
    pi = np.asarray(pi, dtype=np.int64)
    pj = np.asarray(pj, dtype=np.int64)
    nodes, inv = np.unique(np.concatenate([pi, pj]), return_inverse=True)
    pa = np.ascontiguousarray(inv[:pi.size], dtype=np.int32)
    pb = np.ascontiguousarray(inv[pi.size:], dtype=np.int32)
    X, l1, lam, bins = spectra(x, cfg, nodes=nodes)
    Xre = np.ascontiguousarray(X.real)
    Xim = np.ascontiguousarray(X.imag)
    L, B = X.shape[2], X.shape[3]
    npairs = pi.size
    if delta is None:
        delta = DELTA_F64 if cfg.get("elem", "f32") == "f64" else DELTA_F32
    per_bin = np.empty((npairs, B, 7))
    band = np.empty((npairs, 7))
    G = np.empty((npairs, B), dtype=np.int32)
    ties = np.empty((npairs, B), dtype=np.int32)
    sums = np.empty((npairs, B, 8)) if with_sums else None
    aqt = np.empty((npairs, B, 3))
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    lib.orc_pairs(_ptr(Xre), _ptr(Xim), _ptr(l1), K, nodes.size, L, B, _ptr(lam), _ptr(pa),
                  _ptr(pb), npairs, float(delta), _ptr(per_bin), _ptr(band), _ptr(G), _ptr(ties),
                  _ptr(sums) if with_sums else None, _ptr(aqt))
    out = dict(K=K, bins=bins, pi=pi, pj=pj, G=G, ties=ties, A=aqt[:, :, 0], Q=aqt[:, :, 1],
               tsum=aqt[:, :, 2],
               band={m: band[:, q] for q, m in enumerate(METRICS7)},
               per_bin={m: per_bin[:, :, q] for q, m in enumerate(METRICS7)})
    if with_sums:
        out["sums"] = sums
    if with_cor:
        out["band"]["cor"] = cor(x, pi, pj)
    return out


class Sliding:
    """The incremental method on the CPU (throughput baseline; its networks
    are pinned to network() by the CPU tests): running FP64 sums of pairs
    (pi, pj) over a window of W trials, one push at a time."""

    def __init__(self, cfg: dict, N: int, pi, pj, W: int):
        self.cfg, self.N, self.W = cfg, N, W
        self.pi = np.asarray(pi, dtype=np.int64)
        self.pj = np.asarray(pj, dtype=np.int64)
        self.nodes, inv = np.unique(np.concatenate([self.pi, self.pj]), return_inverse=True)
        self.pa = np.ascontiguousarray(inv[:self.pi.size], dtype=np.int32)
        self.pb = np.ascontiguousarray(inv[self.pi.size:], dtype=np.int32)
        self.window = []          # spectra (re, im) of the trials in the window, oldest first
        self.psd = None
        self.state = None
        self.band = None

    def push(self, xk: np.ndarray):
        """xk: [N][M] float64 trial."""
        X, _, lam, _ = spectra(np.ascontiguousarray(xk[None], dtype=np.float64), self.cfg, nodes=self.nodes)
        Xre = np.ascontiguousarray(X[0].real)
        Xim = np.ascontiguousarray(X[0].imag)
        nn, L, B = X.shape[1], X.shape[2], X.shape[3]
        if self.state is None:
            self.psd = np.zeros((nn, B))
            self.state = np.zeros((self.pa.size, B, 7))
            self.band = np.empty((self.pa.size, 7))
        self.window.append((Xre, Xim))
        old = self.window.pop(0) if len(self.window) > self.W else None
        K = len(self.window)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        ore, oim = old if old is not None else (Xre, Xim)
        import time
        t0 = time.perf_counter()
        _load().orc_slide(_ptr(Xre), _ptr(Xim), _ptr(ore), _ptr(oim), int(old is not None), nn, L, B, _ptr(lam),
                          _ptr(self.pa), _ptr(self.pb), self.pa.size, K, _ptr(self.psd), _ptr(self.state),
                          _ptr(self.band))
        self.last_update_s = time.perf_counter() - t0     # the running-sum update alone
        return {m: self.band[:, q] for q, m in enumerate(METRICS7)}


def cor(x: np.ndarray, pi, pj) -> np.ndarray:
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    K, N, M = x.shape
    a = np.ascontiguousarray(pi, dtype=np.int32)
    b = np.ascontiguousarray(pj, dtype=np.int32)
    out = np.empty(a.size)
    lib.orc_cor(_ptr(x), K, N * M, M, M, _ptr(a), _ptr(b), a.size, _ptr(out))
    return out


def xcor(x: np.ndarray, pi, pj, max_lag: int | None = None, with_lag: bool = False):
    """Trial-averaged maximum cross-correlation of pairs (pi, pj) over the
    lags -L..L (L = max_lag, default M-1); see orc_xcor.  x: [K][N][M].
    with_lag: also the lag of the maximum in the last trial (positive: the
    first node advanced against the second)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    K, N, M = x.shape
    L = M - 1 if max_lag is None else int(max_lag)
    a = np.ascontiguousarray(pi, dtype=np.int32)
    b = np.ascontiguousarray(pj, dtype=np.int32)
    out = np.empty(a.size)
    lag = np.empty(a.size, dtype=np.int32)
    lib.orc_xcor(_ptr(x), K, N * M, M, M, L, _ptr(a), _ptr(b), a.size, _ptr(out), _ptr(lag))
    return (out, lag) if with_lag else out


def as_device_input(x: np.ndarray, cfg: dict) -> np.ndarray:
    """The input values the device sees, in float64: float32-rounded unless
    the session computes in float64."""
    if cfg.get("elem", "f32") == "f64":
        return np.asarray(x, dtype=np.float64)
    return np.asarray(x, dtype=np.float32).astype(np.float64)


class use_library:
    """Context manager that points the oracle at another build of oracle.c
    (used by the mutation tests, which compile deliberately broken copies)."""

    def __init__(self, path: str):
        self.path = path
        self.saved = None

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = None
        saved_path = globals()["_LIB"]
        globals()["_LIB"] = self.path
        try:
            _load()
        finally:
            globals()["_LIB"] = saved_path
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False
