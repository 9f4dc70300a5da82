"""Time-resolved phase-connectivity oracle (test infrastructure only): the
analytic-signal approach that the paper sets against its own in Sec. 4 --
restrict every node to a narrow band with a temporal filter, form the
analytic signal with the Hilbert transform, and estimate connectivity from
the instantaneous phase and amplitude, here over windows of samples within a
segment instead of over trials.

Plain FP64 definitions, in this order:

  filter    y = h * x, the full causal convolution of the zero-extended
            segment x[0..M-1] with the FIR h[0..T-1] (length M + T - 1)
  analytic  over F points (the smallest power of two >= max(M + T - 1, 256),
            zero padded):
              Y = DFT_F(y),  Z[k] = m[k] Y[k],
              m[0] = m[F/2] = 1,  m[k] = 2 for 0 < k < F/2,  m[k] = 0 above,
              z[n] = IDFT_F(Z)[n + D],  n = 0..M-1,  D = (T-1)/2
            so Re z is the delay-compensated filtered segment and Im z its
            discrete Hilbert transform
  windows   starts 0, hop, 2 hop, ... while start + len <= M
  metrics   per window and pair i < j, the seven spectral metrics of the
            supplementary metric section with the window's samples in the
            role of the trials: the instantaneous cross-spectrum
            z_i(t) conj(z_j(t)) and the powers |z_i(t)|^2 (the oracle's own
            orc_pairs with one bin and one taper)

Readings: the paper does not fix the filter, the transform length, the edge
handling or the averaging axis of this approach; the definitions above are
the textbook ones (they match scipy.signal.hilbert on the zero-padded full
convolution, which pins them).  The transform is at least 256 points long:
any length >= M + T - 1 gives the analytic signal of the zero-extended
filtered segment, a longer one with a finer-sampled spectrum, so the length
is part of the definition and fixed here.
"""
from __future__ import annotations

import numpy as np

from . import DELTA_F32, METRICS7, _load, _ptr, all_pairs


def fft_len(M: int, T: int) -> int:
    n = M + T - 1
    F = 256
    while F < n:
        F *= 2
    return F


def analytic(x: np.ndarray, h: np.ndarray, F: int | None = None) -> np.ndarray:
    """x: [C][M] real segment; h: [T] taps (odd T).  Returns z [C][M]."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    h = np.asarray(h, dtype=np.float64)
    C, M = x.shape
    T = h.size
    assert T % 2 == 1
    D = (T - 1) // 2
    F = fft_len(M, T) if F is None else int(F)
    assert F >= M + T - 1
    y = np.stack([np.convolve(xc, h) for xc in x])           # [C][M + T - 1]
    Y = np.fft.fft(y, F, axis=1)
    m = np.zeros(F)
    m[0] = 1.0
    m[1:F // 2] = 2.0
    m[F // 2] = 1.0
    z = np.fft.ifft(Y * m[None, :], axis=1)
    return z[:, D:D + M]


def window_starts(M: int, win_len: int = 0, hop: int = 0) -> list[int]:
    L = M if win_len <= 0 else int(win_len)
    H = L if hop <= 0 else int(hop)
    return list(range(0, M - L + 1, H))


def tie_scale(x: np.ndarray, F: int) -> np.ndarray:
    """Per-node scale of the FP32 error of z (||x||_2 2 log2 F / sqrt F): a
    sample whose |Im z_i conj z_j| is within DELTA_F32 (scale_i |z_j| +
    scale_j |z_i|) counts as a tie whose sign the device may take either way."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    return np.sqrt(np.sum(x * x, axis=1)) * 2.0 * np.log2(F) / np.sqrt(F)


def network(z: np.ndarray, win_len: int = 0, hop: int = 0, pi=None, pj=None, scale=None,
            delta: float = DELTA_F32) -> list[dict]:
    """Per window: dict(K, start, band={metric: [np]}, G, ties, A, Q, tsum)
    for pairs (pi, pj) (default every pair i < j in packed order)."""
    lib = _load()
    z = np.atleast_2d(np.asarray(z, dtype=np.complex128))
    N, M = z.shape
    if pi is None:
        pi, pj = all_pairs(N)
    pa = np.ascontiguousarray(pi, dtype=np.int32)
    pb = np.ascontiguousarray(pj, dtype=np.int32)
    npairs = pa.size
    sc = np.zeros(N) if scale is None else np.asarray(scale, dtype=np.float64)
    lam = np.ones(1)
    res = []
    for a in window_starts(M, win_len, hop):
        K = M if win_len <= 0 else int(win_len)
        zw = z[:, a:a + K].T                                  # [K][N] = [K][nn][L=1][B=1]
        Xre = np.ascontiguousarray(zw.real)
        Xim = np.ascontiguousarray(zw.imag)
        l1 = np.ascontiguousarray(np.broadcast_to(sc[None, :], (K, N)))
        per_bin = np.empty((npairs, 1, 7))
        band = np.empty((npairs, 7))
        G = np.empty((npairs, 1), dtype=np.int32)
        ties = np.empty((npairs, 1), dtype=np.int32)
        aqt = np.empty((npairs, 1, 3))
        lib.orc_pairs(_ptr(Xre), _ptr(Xim), _ptr(l1), K, N, 1, 1, _ptr(lam), _ptr(pa), _ptr(pb), npairs,
                      float(delta), _ptr(per_bin), _ptr(band), _ptr(G), _ptr(ties), None, _ptr(aqt))
        res.append(dict(K=K, start=a, G=G, ties=ties, A=aqt[:, :, 0], Q=aqt[:, :, 1], tsum=aqt[:, :, 2],
                        band={m: band[:, q] for q, m in enumerate(METRICS7)}))
    return res
