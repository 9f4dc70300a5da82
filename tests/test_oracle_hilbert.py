"""Pins of the time-resolved analytic-signal oracle (oracle/hilbert.py): the
analytic signal against scipy.signal.hilbert of the zero-padded full
convolution, its real part against the filtered segment, exact closed forms
(a periodic complex exponential, DC and Nyquist), a filtered sinusoid's
instantaneous amplitude and phase, window starts, constant-lag closed forms
per window, a pure-Python brute force with Vinck's pairwise forms, and
planted mistakes that these pins must catch."""
import math
import types

import numpy as np
import pytest
import scipy.signal as sig

import oracle
from oracle import hilbert as oh
from oracle import stream as so


def _h(T=101, fs=1000.0, f1=8.0, f2=30.0):
    return so.fir_design(so.BANDPASS, fs, f1, f2, n_taps=T)


def test_analytic_matches_scipy_hilbert(mod=oh):
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 300))
    for T in (1, 101, 251):
        h = np.ones(1) if T == 1 else _h(T)
        F = mod.fft_len(300, T)
        D = (T - 1) // 2
        z = mod.analytic(x, h)
        ref = np.stack([sig.hilbert(np.convolve(xc, h), N=F)[D:D + 300] for xc in x])
        assert np.allclose(z, ref, atol=1e-12, rtol=0), T
        assert np.allclose(z.real, np.stack([np.convolve(xc, h)[D:D + 300] for xc in x]), atol=1e-12, rtol=0)
        # the filtered segment is the causal filter output advanced by D
        y = sig.lfilter(h, [1.0], np.concatenate([x, np.zeros((3, D))], axis=1), axis=1)[:, D:]
        assert np.allclose(z.real, y, atol=1e-12, rtol=0)


def test_periodic_exponential_is_exact(mod=oh):
    F = 256
    n = np.arange(F)
    for k0, ph in ((5, 0.3), (17, -1.2), (127, 2.0)):
        x = np.cos(2 * np.pi * k0 * n / F + ph)
        z = mod.analytic(x[None, :], np.ones(1))[0]
        assert np.allclose(z, np.exp(1j * (2 * np.pi * k0 * n / F + ph)), atol=1e-12, rtol=0), k0
    for x in (np.full(F, 0.7), 0.7 * np.cos(np.pi * n)):        # DC and Nyquist: the real signal itself
        z = mod.analytic(x[None, :], np.ones(1))[0]
        assert np.allclose(z, x, atol=1e-12, rtol=0)


def test_filtered_sinusoid_amplitude_and_phase(mod=oh):
    fs, M, T, f0, ph = 1000.0, 3000, 251, 19.0, 0.4
    h = _h(T)
    t = np.arange(M) / fs
    z = mod.analytic(np.cos(2 * np.pi * f0 * t + ph)[None, :], h)[0]
    gain = abs(np.sum(h * np.exp(-2j * np.pi * f0 / fs * (np.arange(T) - (T - 1) / 2))))
    mid = slice(1000, 2000)
    assert np.allclose(np.abs(z[mid]), gain, atol=2e-3)
    dphi = np.angle(z[mid] * np.exp(-1j * (2 * np.pi * f0 * t[mid] + ph)))
    assert np.max(np.abs(dphi)) < 2e-3


def test_window_starts(mod=oh):
    assert mod.window_starts(10, 4, 3) == [0, 3, 6]
    assert mod.window_starts(10, 0, 0) == [0]
    assert mod.window_starts(10, 5, 0) == [0, 5]
    assert mod.window_starts(10, 10, 1) == [0]
    assert mod.window_starts(9, 2, 7) == [0, 7]


def test_constant_lag_closed_forms_per_window(mod=oh):
    rng = np.random.default_rng(1)
    M, L, H = 120, 40, 40
    thetas = [0.7, -1.9, 2.5]
    amp = rng.uniform(0.5, 2.0, M)
    phase = np.cumsum(rng.uniform(0.05, 0.3, M))
    za = amp * np.exp(1j * phase)
    zb = np.concatenate([za[w * L:(w + 1) * L] * np.exp(-1j * th) for w, th in enumerate(thetas)])
    noise = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    res = mod.network(np.stack([za, zb, noise]), L, H, pi=[0], pj=[1])
    assert [r["start"] for r in res] == [0, 40, 80]
    for r, th in zip(res, thetas):
        b = r["band"]
        for m in ("coh", "plv", "pli", "wpli", "uspli", "dswpli"):
            assert b[m][0] == pytest.approx(1.0, abs=1e-12), (m, th)
        assert b["imcoh"][0] == pytest.approx(math.sin(th), abs=1e-12)
        assert r["G"][0, 0] == (L if math.sin(th) > 0 else -L)


def _brute(z, i, j, a, K):
    """Metrics of pair (i, j) over samples a..a+K-1, plain loops; USPLI and
    DSWPLI in the pairwise form."""
    cs = [z[i][t] * z[j][t].conjugate() for t in range(a, a + K)]
    pi_ = sum(abs(z[i][t]) ** 2 for t in range(a, a + K))
    pj_ = sum(abs(z[j][t]) ** 2 for t in range(a, a + K))
    S = sum(cs)
    den = math.sqrt(pi_ * pj_)
    ims = [c.imag for c in cs]
    sg = [1 if v > 0 else (-1 if v < 0 else 0) for v in ims]
    out = dict(coh=abs(S) / den, imcoh=S.imag / den, plv=abs(sum(c / abs(c) for c in cs)) / K,
               pli=abs(sum(sg)) / K, wpli=abs(sum(ims)) / sum(abs(v) for v in ims))
    num = sum(sg[p] * sg[q] for p in range(K) for q in range(K) if p != q)
    out["uspli"] = num / (K * (K - 1))
    num = sum(ims[p] * ims[q] for p in range(K) for q in range(K) if p != q)
    den2 = sum(abs(ims[p]) * abs(ims[q]) for p in range(K) for q in range(K) if p != q)
    out["dswpli"] = num / den2
    return out


@pytest.mark.parametrize("L,H", [(0, 0), (5, 3), (7, 7)])
def test_brute_force_tiny(L, H, mod=oh):
    rng = np.random.default_rng(2 + L)
    N, M = 4, 17
    x = rng.standard_normal((N, M)) + 0.3 * rng.standard_normal((1, M))
    z = mod.analytic(x, _h(9))
    res = mod.network(z, L, H)
    pi, pj = oracle.all_pairs(N)
    zl = [[complex(v) for v in row] for row in z]
    K = M if L == 0 else L
    assert len(res) == len(mod.window_starts(M, L, H)) and all(r["K"] == K for r in res)
    for r in res:
        for p in range(pi.size):
            want = _brute(zl, int(pi[p]), int(pj[p]), r["start"], K)
            for m, v in want.items():
                assert r["band"][m][p] == pytest.approx(v, abs=1e-12), (m, p, r["start"])


# ---------------------------------------------------------------- mutants
MUTANTS = [
    ("nyquist_doubled", "m[F // 2] = 1.0", "m[F // 2] = 2.0"),
    ("dc_doubled", "m[0] = 1.0", "m[0] = 2.0"),
    ("negative_kept", "m[1:F // 2] = 2.0", "m[1:F // 2] = 1.0; m[F // 2 + 1:] = 1.0"),
    ("delay_not_compensated", "return z[:, D:D + M]", "return z[:, :M]"),
    ("window_last_dropped", "range(0, M - L + 1, H)", "range(0, M - L, H)"),
    ("window_len_is_hop", "K = M if win_len <= 0 else int(win_len)", "K = M if win_len <= 0 else int(hop or win_len)"),
    ("conjugate_side", "zw = z[:, a:a + K].T", "zw = np.conj(z[:, a:a + K].T)"),
]


def _mutant(orig, mut):
    src = open(oh.__file__).read()
    assert src.count(orig) == 1, orig
    mod = types.ModuleType("oracle.hilbert_mutant")
    mod.__package__ = "oracle"
    exec(compile(src.replace(orig, mut), "hilbert_mutant.py", "exec"), mod.__dict__)
    return mod


def _window_len_mutant_check(mod):
    # windows of 5 with hop 3 must hold 5 samples each
    test_brute_force_tiny(5, 3, mod=mod)


CHECKS = [test_analytic_matches_scipy_hilbert, test_periodic_exponential_is_exact, test_window_starts,
          test_constant_lag_closed_forms_per_window, _window_len_mutant_check,
          lambda mod: test_brute_force_tiny(0, 0, mod=mod)]


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, orig, mut):
    mod = _mutant(orig, mut)
    caught = 0
    for chk in CHECKS:
        try:
            chk(mod=mod)
        except (AssertionError, IndexError, ValueError):
            caught += 1
    assert caught > 0, name
