"""Network post-processing on the device (fcx_network_select) against the
oracle (oracle/netsel.py) on the same FP32 network: the maximum, the
threshold, k, the selected set, the degrees and the normalised weights are
compared bit for bit; strengths (FP64 sums in another order) to 1e-6
relative."""
import numpy as np
import pytest

import synth
from gpu_helpers import log, run_pushes
from oracle import netsel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fcx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2303_03279_amd as m
    return m


def _run(fcx, w_dev, N, fraction, in_place=False):
    import torch
    P = N * (N - 1) // 2
    w_norm = w_dev if in_place else torch.empty(P, dtype=torch.float32, device="cuda")
    sel = torch.empty(P, dtype=torch.uint8, device="cuda")
    deg = torch.empty(N, dtype=torch.int32, device="cuda")
    stren = torch.empty(N, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    st, info = fcx.network_select(N, w_dev.data_ptr(), fraction, w_norm.data_ptr(), sel.data_ptr(),
                                  deg.data_ptr(), stren.data_ptr())
    fcx.check(st, "network_select")
    return info, w_norm.cpu().numpy(), sel.cpu().numpy().astype(bool), deg.cpu().numpy(), stren.cpu().numpy()


def _compare(fcx, w, N, fraction, in_place=False, label=""):
    import torch
    ref = netsel.network_select(w, N, fraction)
    w_dev = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda()
    info, w_norm, sel, deg, stren = _run(fcx, w_dev, N, fraction, in_place)
    assert info["k"] == ref["k"] and info["n_finite"] == ref["n_finite"], label
    assert np.float32(info["max_abs"]) == np.float32(ref["max_abs"]), label
    assert np.float32(info["threshold"]) == np.float32(ref["threshold"]), label
    assert info["n_selected"] == ref["n_selected"], label
    assert np.array_equal(sel, ref["selected"]), label
    assert np.array_equal(deg, ref["degree"]), label
    assert np.array_equal(w_norm, ref["w_norm"], equal_nan=True), label
    assert np.allclose(stren, ref["strength"], rtol=1e-6, atol=1e-30), label
    log(f"netsel {label}: N={N} f={fraction} k={info['k']} selected={info['n_selected']} "
        f"max={info['max_abs']:.6g} T={info['threshold']:.6g}")


def test_session_networks(fcx):
    """coh (non-negative) and imcoh (signed) networks of a live session,
    read on the device, at the paper's 5% and 10% display fractions."""
    import torch
    N = 300
    cfg = synth.base_config(n_nodes=N, n_samples=500, window_trials=12, n_fft=512, f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.COH | synth.IMCOH | synth.USPLI)
    x = synth.source_space(21, N, 12, 500, 12).astype(np.float32)
    s = run_pushes(fcx, cfg, x)
    P = N * (N - 1) // 2
    for metric in ["coh", "imcoh"]:
        out = torch.empty(P, dtype=torch.float32, device="cuda")
        fcx.check(s.read_device(metric, out.data_ptr(), P))
        torch.cuda.synchronize()
        w = out.cpu().numpy()
        for f in (0.05, 0.10):
            _compare(fcx, w, N, f, label=f"session {metric}")
    s.close()


@pytest.mark.parametrize("N", [2, 3, 65, 129, 1000])
def test_random_with_ties_and_nans(fcx, N):
    rng = np.random.default_rng(N)
    P = N * (N - 1) // 2
    w = rng.uniform(-1, 1, P).astype(np.float32)
    w = np.round(w * 64) / 64                      # many exact ties
    if P > 4:
        w[rng.integers(P, size=3)] = np.nan
        w[rng.integers(P)] = -np.inf
    for f in (0.0, 1e-6, 0.05, 0.5, 1.0):
        _compare(fcx, w.astype(np.float32), N, f, label="random ties")
    _compare(fcx, w.astype(np.float32), N, 0.2, in_place=True, label="in place")


def test_degenerate(fcx):
    N = 50
    P = N * (N - 1) // 2
    _compare(fcx, np.zeros(P, dtype=np.float32), N, 0.1, label="all zero")
    _compare(fcx, np.full(P, np.nan, dtype=np.float32), N, 0.1, label="all NaN")
    _compare(fcx, np.full(P, -0.5, dtype=np.float32), N, 0.1, label="all equal")


def test_full_source_size(fcx):
    """5000 nodes (12.5M edges), the size of the source-space networks."""
    N = 5000
    P = N * (N - 1) // 2
    rng = np.random.default_rng(5)
    w = rng.beta(2, 5, P).astype(np.float32)
    _compare(fcx, w, N, 0.05, label="N=5000")
