"""Stream front-end oracle (test infrastructure only): the temporal filter and
the trial cutting that feed pushes from a continuous multichannel stream
(the noise-reduction and averaging plug-ins of the online pipeline, Sec. 2.5).

Written as plain definitions in FP64:

  FIR design (windowed sinc, linear phase, odd length T, centre D = (T-1)/2):
    lowpass(fc)   h[n] = 2 fc/fs sinc(2 fc/fs (n - D)) w[n], scaled to DC gain 1
    highpass(fc)  delta[n - D] - lowpass(fc)[n]  (before windowing: the
                  spectral inversion of the ideal lowpass), scaled to gain 1
                  at Nyquist
    bandpass(f1, f2)  lowpass(f2) - lowpass(f1) (ideal), scaled to gain 1 at
                  the centre frequency (f1 + f2) / 2
    w = Hamming 0.54 - 0.46 cos(2 pi n / (T - 1)); T from the transition
    width dF when not given: T = the odd number >= 3.3 fs / dF
  filtering      y[n] = sum_k h[k] x[n - k] over the whole stream (causal;
                 x = 0 before the first sample), so y lags x by D samples
  events         a rising edge of the trigger channel at sample n when
                 trig[n - 1] < threshold <= trig[n] (trig[-1] = -inf)
  trials         for an event at n0: the filtered data channels at
                 n0 - pre + D .. n0 + post - 1 + D, i.e. the samples of raw
                 time n0 - pre .. n0 + post - 1, once all are available;
                 an event whose window starts before the stream is dropped.

Readings: the paper names the design parameters (cutoffs, transition
bandwidth, method, taps) and the FFT overlap-add realisation but no design
formula; the Hamming windowed sinc with these scalings is the textbook
method (it matches scipy.signal.firwin, which pins it).
"""
from __future__ import annotations

import math

import numpy as np

LOWPASS, HIGHPASS, BANDPASS = 0, 1, 2


def taps_for(fs: float, transition_hz: float) -> int:
    T = int(math.ceil(3.3 * fs / transition_hz))
    return T if T % 2 == 1 else T + 1


def fir_design(kind: int, fs: float, f1: float, f2: float = 0.0, transition_hz: float = 0.0, n_taps: int = 0):
    T = n_taps if n_taps > 0 else taps_for(fs, transition_hz)
    assert T % 2 == 1 and T >= 3
    D = (T - 1) / 2.0
    n = np.arange(T, dtype=np.float64)
    w = 0.54 - 0.46 * np.cos(2.0 * np.pi * n / (T - 1))

    def ideal_lp(fc):
        return 2.0 * fc / fs * np.sinc(2.0 * fc / fs * (n - D))

    if kind == LOWPASS:
        h = ideal_lp(f1) * w
        f0 = 0.0
    elif kind == HIGHPASS:
        h = (np.where(n == D, 1.0, 0.0) - ideal_lp(f1)) * w
        f0 = fs / 2.0
    elif kind == BANDPASS:
        h = (ideal_lp(f2) - ideal_lp(f1)) * w
        f0 = (f1 + f2) / 2.0
    else:
        raise ValueError(kind)
    g = np.sum(h * np.cos(2.0 * np.pi * f0 / fs * (n - D)))
    return h / g


def filter_stream(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Causal FIR over the whole stream, x: [C][n] -> y: [C][n]."""
    x = np.asarray(x, dtype=np.float64)
    return np.stack([np.convolve(xc, h)[:x.shape[1]] for xc in x])


def events(trig: np.ndarray, threshold: float) -> np.ndarray:
    t = np.asarray(trig, dtype=np.float64)
    prev = np.concatenate([[-np.inf], t[:-1]])
    return np.flatnonzero((prev < threshold) & (t >= threshold))


def cut_trials(y: np.ndarray, ev, pre: int, post: int, D: int):
    """Trials [K][C][pre+post] from the filtered stream y for the events ev
    whose window lies inside the stream; returns (trials, kept events)."""
    n = y.shape[1]
    out, kept = [], []
    for n0 in ev:
        a, b = n0 - pre + D, n0 + post + D
        if n0 - pre < 0 or b > n:
            continue
        out.append(y[:, a:b])
        kept.append(int(n0))
    if not out:
        return np.zeros((0, y.shape[0], pre + post)), np.array(kept, dtype=np.int64)
    return np.stack(out), np.array(kept, dtype=np.int64)
