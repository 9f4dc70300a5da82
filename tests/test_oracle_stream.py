"""Pins of the stream front-end oracle (oracle/stream.py): the FIR design
against scipy.signal.firwin, frequency responses at DC / Nyquist / the band
centre, linear phase (symmetric taps); the filter against
scipy.signal.lfilter; events and trial windows against explicit loops."""
import numpy as np
import pytest
import scipy.signal as sig

from oracle import stream as so


@pytest.mark.parametrize("kind,f1,f2,T", [(so.LOWPASS, 40.0, 0.0, 101), (so.HIGHPASS, 2.0, 0.0, 401),
                                          (so.HIGHPASS, 20.0, 0.0, 401), (so.BANDPASS, 8.0, 30.0, 251),
                                          (so.LOWPASS, 100.0, 0.0, 31)])
def test_design_matches_firwin(kind, f1, f2, T):
    fs = 1000.0
    h = so.fir_design(kind, fs, f1, f2, n_taps=T)
    if kind == so.LOWPASS:
        ref = sig.firwin(T, f1, window="hamming", pass_zero=True, fs=fs)
    elif kind == so.HIGHPASS:
        ref = sig.firwin(T, f1, window="hamming", pass_zero=False, fs=fs)
    else:
        ref = sig.firwin(T, [f1, f2], window="hamming", pass_zero=False, fs=fs)
    assert np.allclose(h, ref, atol=1e-14, rtol=0)
    assert np.allclose(h, h[::-1], atol=1e-15)                       # linear phase
    H = np.fft.rfft(h, 1 << 16)
    f = np.fft.rfftfreq(1 << 16, 1 / fs)
    if kind == so.LOWPASS:
        assert abs(H[0]) == pytest.approx(1.0, abs=1e-12)
    elif kind == so.HIGHPASS:
        assert abs(H[-1]) == pytest.approx(1.0, abs=1e-12)
        if f1 > 3.3 * fs / T:               # cutoff above the transition width: DC is stopped
            assert abs(H[0]) < 1e-2
    else:
        assert abs(H[np.argmin(np.abs(f - 19.0))]) == pytest.approx(1.0, abs=1e-2)


def test_taps_from_transition():
    assert so.taps_for(1000.0, 10.0) == 331
    assert so.taps_for(1000.0, 33.0) == 101
    assert len(so.fir_design(so.LOWPASS, 1000.0, 40.0, transition_hz=10.0)) == 331


def test_filter_matches_lfilter():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 1000))
    h = so.fir_design(so.BANDPASS, 1000.0, 8.0, 30.0, n_taps=151)
    assert np.allclose(so.filter_stream(x, h), sig.lfilter(h, [1.0], x, axis=1), atol=1e-12, rtol=0)


def test_events_and_trials():
    trig = np.zeros(100)
    trig[[10, 11, 12, 40, 97]] = 5.0      # edges at 10, 40, 97 (11, 12 stay high)
    trig[70] = 0.5                        # below threshold
    ev = so.events(trig, 1.0)
    assert list(ev) == [10, 40, 97]
    assert list(so.events(np.full(5, 3.0), 1.0)) == [0]    # high from the start: an edge at 0
    y = np.arange(2 * 100, dtype=float).reshape(2, 100)
    tr, kept = so.cut_trials(y, ev, pre=5, post=10, D=3)
    assert list(kept) == [10, 40]                           # 97 + 10 + 3 > 100: not yet complete
    assert np.array_equal(tr[0], y[:, 10 - 5 + 3:10 + 10 + 3])
    tr, kept = so.cut_trials(y, ev, pre=12, post=10, D=3)
    assert list(kept) == [40]                               # 10 - 12 < 0: before the stream
