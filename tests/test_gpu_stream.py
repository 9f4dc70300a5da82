"""Stream front end on the device (fcx_stream_*) against the oracle
(oracle/stream.py): the block-filtered stream equals the causal FIR over the
whole stream (overlap-add across blocks, tails longer than a block), events
and trial windows are exact, trial samples within the FP32 FFT error; and
trials cut on the device feed a session whose network matches the oracle's
network of the oracle's trials."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, compare_network, log
from oracle import stream as so

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fcx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2303_03279_amd as m
    return m


def _stream_input(seed, C, n, fs, ev_at):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((C, n)).astype(np.float32)
    t = np.arange(n) / fs
    x += (2.0 * np.sin(2 * np.pi * 20.0 * t))[None, :].astype(np.float32)   # in band
    x += (3.0 * np.sin(2 * np.pi * 150.0 * t))[None, :].astype(np.float32)  # out of band
    trig = np.zeros(n, dtype=np.float32)
    for e in ev_at:
        trig[e:e + 5] = 4.0
    return x, trig


def _run(fcx, x, trig, block, taps, pre, post, thr=1.0, cap=16):
    import torch
    C, n = x.shape
    s = fcx.Stream(C, block, taps, thr, pre, post)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(trig).cuda()
    y = torch.empty((C, block), dtype=torch.float32, device="cuda")
    tr = torch.empty((cap, C, pre + post), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    ys, trials, dropped = [], [], 0
    for b0 in range(0, n - block + 1, block):
        st, k, d = s.push(xd.data_ptr() + 4 * b0, n, td.data_ptr() + 4 * b0, y.data_ptr(), tr.data_ptr(), cap)
        fcx.check(st, "stream push")
        ys.append(y.cpu().numpy().copy())
        trials.extend(tr[:k].cpu().numpy().copy())
        dropped += d
    fcx.check(s.close())
    return np.concatenate(ys, axis=1), np.array(trials), dropped


@pytest.mark.parametrize("C,block,T,pre,post", [(7, 100, 101, 30, 120), (6, 500, 251, 100, 400),
                                                (3, 64, 301, 0, 50)])
def test_filter_and_trials_vs_oracle(fcx, C, block, T, pre, post):
    fs = 1000.0
    n = block * (4000 // block)
    ev = [20, 333, 1499, 2001, 2002 + 7, 3600, n - 40]   # one before pre, one at the end (incomplete)
    x, trig = _stream_input(C + block, C, n, fs, ev)
    taps = so.fir_design(so.BANDPASS, fs, 8.0, 30.0, n_taps=T)
    y, trials, dropped = _run(fcx, x, trig, block, taps, pre, post)
    yref = so.filter_stream(x.astype(np.float64), taps)
    scale = np.max(np.abs(yref))
    err = np.max(np.abs(y - yref)) / scale
    D = (T - 1) // 2
    evr = so.events(trig, 1.0)
    tref, kept = so.cut_trials(yref, evr, pre, post, D)
    log(f"stream C={C} block={block} T={T}: filtered max rel err {err:.2e}; events {list(evr)}, "
        f"trials {len(trials)} (oracle {len(kept)}), dropped {dropped}")
    assert err <= TOL
    assert len(trials) == len(kept)
    assert dropped == sum(1 for e in evr if e - pre < 0)
    if len(kept):
        assert np.max(np.abs(trials - tref)) / scale <= TOL


def test_cut_trials_feed_a_session(fcx):
    """The online pipeline in small: stream -> filter -> trials -> push ->
    network, against the oracle network of the oracle's trials."""
    import torch
    fs, C, block, T, pre, post = 1000.0, 40, 250, 151, 50, 450
    n = 250 * 24
    ev = list(range(300, n - 600, 700))
    x, trig = _stream_input(11, C, n, fs, ev)
    x[5, 40:] += 0.8 * x[4, :-40]
    taps = so.fir_design(so.BANDPASS, fs, 4.0, 45.0, n_taps=T)
    s = fcx.Stream(C, block, taps, 1.0, pre, post)
    cfg = synth.base_config(n_nodes=C, n_samples=pre + post, window_trials=5, n_fft=512, fs_hz=fs, f_lo_hz=8,
                            f_hi_hz=30, metrics=synth.ALL8)
    sess = fcx.Session(cfg)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(trig).cuda()
    tr = torch.empty((8, C, pre + post), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    total = 0
    for b0 in range(0, n - block + 1, block):
        st, k, d = s.push(xd.data_ptr() + 4 * b0, n, td.data_ptr() + 4 * b0, 0, tr.data_ptr(), 8)
        fcx.check(st)
        for q in range(k):
            fcx.check(sess.push_device(tr[q].data_ptr(), pre + post))
        fcx.check(sess.sync())
        total += k
    yref = so.filter_stream(x.astype(np.float64), taps)
    tref, kept = so.cut_trials(yref, so.events(trig, 1.0), pre, post, (T - 1) // 2)
    assert total == len(kept) and total >= 5
    W = cfg["window_trials"]
    ref = oracle.network(tref[-W:].astype(np.float32).astype(np.float64), cfg)
    compare_network(sess, ref, cfg, ["coh", "imcoh", "plv", "wpli", "cor"], label="stream -> session")
    sess.close()
    fcx.check(s.close())
