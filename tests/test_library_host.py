"""Host-side checks of the HIP library that need no GPU: it loads, exports
every symbol the header declares, and its host logic (configuration checks,
band plan, footprint, DPSS) is right."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

fcx = pytest.importorskip("paper_2303_03279_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "fcx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(fcx_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_exports_every_declared_symbol():
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(fcx.lib, n), n
        assert n in fcx.EXPORTED, n


def test_status_strings():
    for st in range(8):
        assert fcx.lib.fcx_status_str(st)
    assert fcx.lib.fcx_status_str(fcx.FCX_E_BUSY).decode() == "HBM budget exhausted"


@pytest.mark.parametrize("F,lo,hi", [(512, 8, 30), (1000, 4, 40), (1024, 8, 30), (256, 0, 500), (600, 8, 12)])
def test_band_plan_matches_oracle(F, lo, hi):
    cfg = synth.base_config(n_nodes=10, n_samples=min(F, 500), window_trials=5, n_fft=F, f_lo_hz=lo, f_hi_hz=hi)
    n, klo, khi = fcx.band_bins(cfg)
    ref = oracle.band_bins(F, 1000.0, lo, hi)
    assert n == ref.size and klo == ref[0] and khi == ref[-1]


def test_invalid_configs_rejected():
    good = synth.base_config(n_nodes=10, n_samples=100, window_trials=5, n_fft=128, f_lo_hz=8, f_hi_hz=30)
    assert fcx.footprint_bytes(good) > 0
    bad = [dict(n_nodes=1), dict(n_samples=1), dict(window_trials=0), dict(n_fft=50),
           dict(fs_hz=0.0), dict(f_lo_hz=40, f_hi_hz=30), dict(metrics=0), dict(metrics=512),
           dict(metrics=synth.XCOR, xcor_max_lag=100), dict(metrics=synth.XCOR, xcor_max_lag=-1),
           dict(metrics=synth.XCOR, n_samples=1500, n_fft=2048),
           dict(taper="dpss", dpss_k=0, dpss_nw=2.0), dict(taper="dpss", dpss_k=3, dpss_nw=60.0)]
    for b in bad:
        cfg = dict(good)
        cfg.update(b)
        assert fcx.footprint_bytes(cfg) == -1, b
    c = fcx.make_config(good)
    c.struct_size = 4
    h = ctypes.c_void_p()
    assert fcx.lib.fcx_open(ctypes.byref(c), None, ctypes.byref(h)) == fcx.FCX_E_INVAL


def test_footprint_scales_with_metrics():
    base = synth.base_config(n_nodes=5000, n_samples=500, window_trials=50, n_fft=512, f_lo_hz=8, f_hi_hz=30)
    all8 = fcx.footprint_bytes(dict(base, metrics=synth.ALL8))
    coh = fcx.footprint_bytes(dict(base, metrics=synth.COH))
    wpli = fcx.footprint_bytes(dict(base, metrics=synth.WPLI))
    # 3160 tiles x 12 bins x 4096 slots: all-8 keeps 4 FP64 planes, 2 int32
    # fixed-point phasor planes and int8 signs (~6.4 GB) plus the COR sample
    # ring, spectra ring and outputs (~1 GB); coh and wpli keep 2 FP64 planes
    slots = 3160 * 12 * 4096
    assert abs(all8 - (slots * (4 * 8 + 2 * 4 + 1) + 1.0e9)) < 0.1e9
    assert 2.4e9 < coh < 3.0e9 and 2.4e9 < wpli < 3.0e9


def test_pair_update_bytes():
    base = synth.base_config(n_nodes=5000, n_samples=500, window_trials=50, n_fft=512, f_lo_hz=8, f_hi_hz=30)
    P, B = 5000 * 4999 // 2, 12
    # all 8: per pair and bin 2 x (4 x 8 + 2 x 4 + 1) bytes; per pair 7 band means,
    # the COR sum read and written and the COR output
    assert fcx.pair_update_bytes(dict(base, metrics=synth.ALL8)) == P * (2 * 41 * B + 7 * 4 + 16 + 4)
    assert fcx.pair_update_bytes(dict(base, metrics=synth.COH)) == P * (2 * 16 * B + 4)
    assert fcx.pair_update_bytes(dict(base, metrics=synth.WPLI)) == P * (2 * 16 * B + 4)
    # long windows keep FP64 phasor sums and int16 signs
    assert fcx.pair_update_bytes(dict(base, metrics=synth.PLV | synth.PLI, window_trials=300)) == \
        P * (2 * 18 * B + 8)


def test_bad_handles():
    h = ctypes.c_void_p(987654321)
    assert fcx.lib.fcx_sync(h) == fcx.FCX_E_INVAL
    assert fcx.lib.fcx_close(h) == fcx.FCX_E_INVAL
    assert fcx.lib.fcx_server_drain(h) == fcx.FCX_E_INVAL


@pytest.mark.parametrize("M,NW,K", [(1000, 2.0, 3), (500, 2.5, 4), (64, 1.5, 2)])
def test_host_dpss_matches_scipy(M, NW, K):
    from scipy.signal.windows import dpss as sp_dpss
    tap, rat = fcx.dpss(M, NW, K)
    ref, rref = sp_dpss(M, NW, K, return_ratios=True)
    assert np.allclose(tap, ref, atol=1e-9)
    assert np.allclose(rat, rref, atol=1e-9)


def test_network_select_rejects_bad_arguments():
    """Argument checks run before any device work (no GPU needed)."""
    st, _ = fcx.network_select(1, 0x1000, 0.1)
    assert st == fcx.FCX_E_INVAL
    st, _ = fcx.network_select(10, 0, 0.1)          # NULL network
    assert st == fcx.FCX_E_INVAL
    for f in (-0.01, 1.5, float("nan")):
        st, _ = fcx.network_select(10, 0x1000, f)
        assert st == fcx.FCX_E_INVAL, f
    st, _ = fcx.network_select(70000, 0x1000, 0.1)
    assert st == fcx.FCX_E_INVAL


def test_xcor_config_and_footprint():
    """XCOR lags -L..L with L <= M - 1 and M + L <= 2048; its buffers: node
    spectra and energies, the per-trial maxima ring and the window sum."""
    base = synth.base_config(n_nodes=300, n_samples=500, window_trials=20, n_fft=512, f_lo_hz=8, f_hi_hz=30,
                             metrics=synth.COH)
    fp = fcx.footprint_bytes(base)
    x = fcx.footprint_bytes(dict(base, metrics=synth.COH | synth.XCOR))
    assert x > fp
    assert fcx.footprint_bytes(dict(base, metrics=synth.XCOR, xcor_max_lag=499)) > 0
    assert fcx.footprint_bytes(dict(base, metrics=synth.XCOR, xcor_max_lag=500)) == -1
    assert fcx.footprint_bytes(dict(base, metrics=synth.XCOR, n_samples=1024, n_fft=1024)) > 0   # 1024+1023 <= 2048
    assert fcx.footprint_bytes(dict(base, metrics=synth.XCOR, n_samples=1025, n_fft=2048)) == -1
    assert fcx.footprint_bytes(dict(base, metrics=synth.XCOR, n_samples=1025, n_fft=2048, xcor_max_lag=1023)) > 0


def test_fir_design_matches_oracle():
    """The library's FIR design (host code) against the oracle's definition."""
    from oracle import stream as so
    for kind, f1, f2, T in [(fcx.FCX_FIR_LOWPASS, 40.0, 0.0, 101), (fcx.FCX_FIR_HIGHPASS, 20.0, 0.0, 401),
                            (fcx.FCX_FIR_BANDPASS, 8.0, 30.0, 251)]:
        got = fcx.fir_design(kind, 1000.0, f1, f2, n_taps=T)
        assert np.allclose(got, so.fir_design(kind, 1000.0, f1, f2, n_taps=T), atol=1e-14, rtol=0)
    assert fcx.fir_design(fcx.FCX_FIR_LOWPASS, 1000.0, 40.0, transition_hz=10.0).size == so.taps_for(1000.0, 10.0)
    n = ctypes.c_int32()
    for args in [(fcx.FCX_FIR_LOWPASS, 1000.0, 600.0, 0.0, 0.0, 101), (fcx.FCX_FIR_BANDPASS, 1000.0, 30.0, 8.0, 0.0, 101),
                 (fcx.FCX_FIR_LOWPASS, 1000.0, 40.0, 0.0, 0.0, 100), (7, 1000.0, 40.0, 0.0, 0.0, 101),
                 (fcx.FCX_FIR_LOWPASS, 1000.0, 40.0, 0.0, 0.0, 0)]:
        assert fcx.lib.fcx_fir_design(*args, None, 0, ctypes.byref(n)) == fcx.FCX_E_INVAL, args


def test_hilbert_rejects_bad_configs():
    """fcx_hilbert_open checks its configuration before any device work; an
    unknown handle is reported as closed."""
    taps = np.ones(5) / 5.0

    def cfg(**kw):
        c = fcx.fcx_hilbert_config()
        c.struct_size = ctypes.sizeof(fcx.fcx_hilbert_config)
        c.n_nodes, c.n_samples, c.n_taps, c.taps = 10, 100, taps.size, taps.ctypes.data
        c.win_len, c.win_hop, c.metrics, c.gram_precision = 0, 0, 0x7F, 0
        for k, v in kw.items():
            setattr(c, k, v)
        return c

    h = ctypes.c_void_p()
    for bad in [dict(n_nodes=1), dict(n_nodes=70000), dict(n_samples=0), dict(n_taps=4), dict(n_taps=0),
                dict(metrics=0), dict(metrics=0x80), dict(metrics=0x100), dict(win_len=101), dict(win_len=-1),
                dict(win_hop=-2), dict(gram_precision=3), dict(n_samples=4000, n_taps=99), dict(taps=None),
                dict(struct_size=4)]:
        assert fcx.lib.fcx_hilbert_open(ctypes.byref(cfg(**bad)), None, ctypes.byref(h)) == fcx.FCX_E_INVAL, bad
    nan_taps = np.array([0.2, np.nan, 0.2])
    c = cfg(n_taps=3, taps=nan_taps.ctypes.data)
    assert fcx.lib.fcx_hilbert_open(ctypes.byref(c), None, ctypes.byref(h)) == fcx.FCX_E_INVAL
    bogus = ctypes.c_void_p(987654321)
    assert fcx.lib.fcx_hilbert_run(bogus, 1, 100, 1, None) == fcx.FCX_E_CLOSED
    assert fcx.lib.fcx_hilbert_info(bogus, None, None) == fcx.FCX_E_CLOSED
    assert fcx.lib.fcx_hilbert_close(bogus) == fcx.FCX_E_CLOSED
