"""One-pass rebuild of the running sums (fcx_resync, and the switch from a
batch pass to sliding pushes) against a session that pushed the same window
into empty sums: the band-mean and per-bin networks of every metric are
bit-identical (the per-bin networks are read straight from the rebuilt sums),
and stay bit-identical while both sessions keep sliding (each evicted trial
cancels exactly what it added).  The rebuilt session is also checked against
the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare_network, log, run_pushes

pytestmark = pytest.mark.gpu

ALL = ["coh", "imcoh", "plv", "pli", "wpli", "uspli", "dswpli", "cor"]
SPECTRAL = ALL[:7]


@pytest.fixture(scope="module")
def fcx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2303_03279_amd as m
    return m


def _case(name):
    if name == "c2":
        x, cfg = synth.c2_sensor(n_trials=150)
        return x, cfg, 140
    rng = np.random.default_rng(17)
    if name == "dpss":
        N, M, W, T = 70, 200, 8, 30
        x = rng.standard_normal((T, N, M))
        x[:, 1, 4:] += 0.9 * x[:, 0, :-4]
        cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=256, f_lo_hz=4, f_hi_hz=120,
                                taper="dpss", dpss_nw=2.0, dpss_k=3, metrics=synth.ALL8)
        return x, cfg, 20
    # FP64 session
    N, M, W, T = 40, 128, 6, 22
    x = rng.standard_normal((T, N, M))
    x[:, 2, 3:] += 0.8 * x[:, 1, :-3]
    cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=128, f_lo_hz=20, f_hi_hz=200,
                            metrics=synth.ALL8, elem="f64")
    return x, cfg, 16


def _networks(s):
    out = {}
    for m in ALL:
        st, v, _ = s.read(m)
        out[m] = v.copy()
        if m in SPECTRAL:
            st, v, _ = s.read(m, per_bin=True)
            out[m + "/bins"] = v.copy()
    return out


def _same(a, b, label):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), (label, k, float(np.nanmax(np.abs(a[k] - b[k]))))


@pytest.mark.parametrize("case", ["c2", "dpss", "f64"])
def test_resync_equals_fresh_window(fcx, case):
    x, cfg, T = _case(case)
    W = cfg["window_trials"]
    log(f"rebuild {case}: N={cfg['n_nodes']} W={W}, {T} pushes then resync")
    a = run_pushes(fcx, cfg, x, 0, T)                     # slid T - W times
    fcx.check(a.resync(), "resync")
    b = run_pushes(fcx, cfg, x, T - W, T)                 # the same window into empty sums
    _same(_networks(a), _networks(b), f"{case} after resync")
    ref = oracle.network(oracle.as_device_input(x[T - W:T], cfg), cfg)
    if cfg.get("elem") == "f64":
        # FP64 session: the spectral metrics in FP64; COR comes from FP32
        # z-scored samples through the FP32 matrix cores in every session
        compare_network(a, ref, cfg, SPECTRAL, tol=1e-11, label=f"{case} resync")
        compare_network(a, ref, cfg, ["cor"], tol=1e-5, label=f"{case} resync cor")
    else:
        compare_network(a, ref, cfg, ALL, label=f"{case} resync")
    run_pushes(fcx, cfg, x, T, x.shape[0], session=a)
    run_pushes(fcx, cfg, x, T, x.shape[0], session=b)
    _same(_networks(a), _networks(b), f"{case} after {x.shape[0] - T} more pushes")
    a.close()
    b.close()


@pytest.mark.parametrize("case", ["c2", "dpss"])
def test_batch_then_slide_equals_fresh_window(fcx, case):
    """A batch pass, then the per-bin read rebuilds the running sums: every
    network equals the fresh session's, before and after more pushes."""
    import torch
    x, cfg, T = _case(case)
    W = cfg["window_trials"]
    N, M = cfg["n_nodes"], cfg["n_samples"]
    c = fcx.Session(cfg)
    xd = torch.from_numpy(np.ascontiguousarray(x[T - W:T], dtype=np.float32)).cuda()
    torch.cuda.synchronize()
    fcx.check(c.push_batch_device(xd.data_ptr(), W, N * M, M), "batch")
    fcx.check(c.sync(), "sync")
    b = run_pushes(fcx, cfg, x, T - W, T)
    fcx.check(c.read("coh", per_bin=True)[0], "per-bin read")   # rebuilds the running sums
    _same(_networks(c), _networks(b), f"{case} batch, rebuilt by the per-bin read")
    run_pushes(fcx, cfg, x, T, x.shape[0], session=c)
    run_pushes(fcx, cfg, x, T, x.shape[0], session=b)
    _same(_networks(c), _networks(b), f"{case} batch then {x.shape[0] - T} pushes")
    c.close()
    b.close()


def test_resync_cor_only(fcx):
    """A session with COR alone (only the COR rebuild runs), ragged tiles and
    a last sample chunk shorter than the others: resync equals the fresh
    window bit for bit, before and after more pushes."""
    rng = np.random.default_rng(23)
    N, M, W, T = 130, 300, 5, 12
    x = rng.standard_normal((T + 3, N, M))
    x[:, 5, 2:] += 0.7 * x[:, 4, :-2]
    cfg = synth.base_config(n_nodes=N, n_samples=M, window_trials=W, n_fft=512, f_lo_hz=8, f_hi_hz=30,
                            metrics=synth.COR)
    log(f"rebuild cor only: N={N} M={M} W={W}")
    a = run_pushes(fcx, cfg, x, 0, T)
    fcx.check(a.resync(), "resync")
    b = run_pushes(fcx, cfg, x, T - W, T)
    assert np.array_equal(a.read("cor")[1], b.read("cor")[1])
    ref = oracle.network(oracle.as_device_input(x[T - W:T], cfg), cfg)
    compare_network(a, ref, cfg, ["cor"], label="cor only resync")
    run_pushes(fcx, cfg, x, T, x.shape[0], session=a)
    run_pushes(fcx, cfg, x, T, x.shape[0], session=b)
    assert np.array_equal(a.read("cor")[1], b.read("cor")[1])
    a.close()
    b.close()
