"""Serving form: continuous batching of many sessions in one device stream.

Each session's networks must be identical (bit for bit) whether it runs
alone through the plain push path or mixed with other sessions in the
server's batched launches, with its queued trials coalesced into one pass
over its running sums; admission must respect the HBM budget; a read waits
for every trial submitted before it."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare_network, log, run_pushes

pytestmark = pytest.mark.gpu

ALL = ["coh", "imcoh", "plv", "pli", "wpli", "uspli", "dswpli", "cor"]


@pytest.fixture(scope="module")
def fcx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2303_03279_amd as m
    return m


def _mix_configs():
    base = dict(n_samples=500, n_fft=512, fs_hz=1000.0, f_lo_hz=8.0, f_hi_hz=30.0)
    return [
        synth.base_config(n_nodes=60, window_trials=10, metrics=synth.ALL8, **base),
        synth.base_config(n_nodes=128, window_trials=7, metrics=synth.COH | synth.PLI, **base),
        synth.base_config(n_nodes=306, window_trials=12, metrics=synth.WPLI | synth.DSWPLI, **base),
        synth.base_config(n_nodes=200, window_trials=5, metrics=synth.COR, **base),
        synth.base_config(n_nodes=97, window_trials=3, metrics=synth.PLV | synth.IMCOH | synth.USPLI, **base),
        # one session of each remaining compile-time kernel class: COH only,
        # WPLI only, three DPSS tapers, 16-bit sign sums (W > 127) and
        # FP64 phasor sums (W > 256)
        synth.base_config(n_nodes=150, window_trials=20, metrics=synth.COH, **base),
        synth.base_config(n_nodes=90, window_trials=8, metrics=synth.WPLI, **base),
        synth.base_config(n_nodes=80, window_trials=6, metrics=synth.ALL8, taper="dpss", dpss_nw=2.0, dpss_k=3,
                          **base),
        synth.base_config(n_nodes=70, window_trials=140, metrics=synth.ALL8, **base),
        synth.base_config(n_nodes=66, window_trials=300, metrics=synth.ALL8 & ~synth.COR, **base),
    ]


def test_alone_equals_mix(fcx):
    cfgs = _mix_configs()
    T = [14, 11, 16, 9, 8, 30, 12, 10, 150, 310]
    xs = [synth.c4_trials(c, 100 + k, T[k]).astype(np.float32) for k, c in enumerate(cfgs)]
    alone = []
    for c, x in zip(cfgs, xs):
        s = run_pushes(fcx, c, x)
        names = [m for m in ALL if c["metrics"] & synth.METRIC_BITS[m]]
        alone.append({m: s.read(m)[1].copy() for m in names})
        s.close()
    srv = fcx.Server(1 << 36)
    sess = []
    for c in cfgs:
        st, ss = srv.open(c)
        fcx.check(st)
        sess.append(ss)
    # interleave submissions across sessions (per-session order preserved);
    # the first 200 are queued while the server is held, so the first ticks
    # coalesce full groups, the rest run as they arrive
    rng = np.random.default_rng(0)
    cursor = [0] * len(cfgs)
    tickets = []
    fcx.check(srv.hold(True))
    while any(cursor[k] < T[k] for k in range(len(cfgs))):
        k = int(rng.integers(len(cfgs)))
        if cursor[k] < T[k]:
            tickets.append(srv.submit(sess[k], np.ascontiguousarray(xs[k][cursor[k]])))
            cursor[k] += 1
            if len(tickets) == 200:
                fcx.check(srv.hold(False))
    srv.drain()
    lat = []
    for t in tickets:
        done, l = srv.poll(t)
        assert done and l > 0
        lat.append(l)
    ticks, trials, group, busy = srv.counts()
    log(f"served {len(tickets)} trials in {ticks} ticks (largest coalesced group {group}), "
        f"latency p50 {1e3 * np.median(lat):.2f} ms")
    assert trials == len(tickets)
    assert group == 8         # the held submissions were coalesced in full groups
    for k, c in enumerate(cfgs):
        for m, ref in alone[k].items():
            st, out, K = sess[k].read(m)
            assert K == min(T[k], c["window_trials"])
            assert np.array_equal(out, ref, equal_nan=True), (k, m)
    # and some of them against the oracle
    for k in (0, 7, 8):
        c, x = cfgs[k], xs[k]
        W = c["window_trials"]
        ref = oracle.network(oracle.as_device_input(x[T[k] - W:], c), c)
        compare_network(sess[k], ref, c, ALL, label=f"served N={c['n_nodes']} W={W} L={c.get('dpss_k', 1)}")
    for ss in sess:
        fcx.check(ss.close())
    fcx.check(srv.destroy())


def _served_bytes(fcx, c):
    # a served session holds the plain session's buffers with 7 more ring
    # slots plus two device input buffers of 8 trials (256-byte aligned)
    N, M, W = c["n_nodes"], c["n_samples"], c["window_trials"]
    xb = (N * M * 4 + 255) // 256 * 256
    spectral = c["metrics"] & 0x7F
    B = fcx.band_bins(c)[0]
    L = c.get("dpss_k", 1) if c.get("taper") == "dpss" else 1
    mz = (M + 31) // 32 * 32
    def al(v):
        return (v + 255) // 256 * 256
    extra = 0
    if spectral:
        extra += al((W + 8) * B * L * N * 8) - al((W + 1) * B * L * N * 8)
    if c["metrics"] & 128:
        extra += al((W + 8) * N * mz * 4) - al((W + 1) * N * mz * 4)
    fp = fcx.footprint_bytes(c) + extra + 2 * 8 * xb
    assert fp == fcx.server_footprint_bytes(c)
    return fp


def test_admission_by_hbm_budget(fcx):
    c = synth.base_config(n_nodes=1000, n_samples=500, window_trials=40, n_fft=512, f_lo_hz=8, f_hi_hz=30,
                          metrics=synth.ALL8)
    fp = _served_bytes(fcx, c)
    srv = fcx.Server(int(1.5 * fp))
    st, a = srv.open(c)
    fcx.check(st)
    used, left, n = srv.usage()
    assert used == fp and n == 1
    st, b = srv.open(c)
    assert st == fcx.FCX_E_BUSY and b is None
    small = dict(c, n_nodes=60)
    st, s2 = srv.open(small)
    fcx.check(st)                               # a smaller session still fits
    assert srv.usage()[0] == fp + _served_bytes(fcx, small)
    x = synth.c4_trials(c, 5, 3).astype(np.float32)
    for k in range(3):
        srv.submit(a, np.ascontiguousarray(x[k]))
    fcx.check(a.close())                        # drains, then frees its memory
    st, b = srv.open(c)
    fcx.check(st)
    assert srv.usage()[0] == fp + _served_bytes(fcx, small)
    fcx.check(b.close())
    fcx.check(s2.close())
    assert srv.usage()[0] == 0
    fcx.check(srv.destroy())


def test_served_nonfinite_rejected(fcx):
    """A non-finite trial in the middle of a burst: the finite ones around it
    are coalesced, it goes alone and is rejected, the window holds the
    accepted trials in order."""
    c = synth.base_config(n_nodes=64, n_samples=500, window_trials=4, n_fft=512, f_lo_hz=8, f_hi_hz=30,
                          metrics=synth.ALL8)
    x = synth.c4_trials(c, 9, 8).astype(np.float32)
    srv = fcx.Server(1 << 34)
    st, s = srv.open(c)
    fcx.check(st)
    for k in range(5):
        srv.submit(s, np.ascontiguousarray(x[k]))
    bad = x[5].copy()
    bad[3, 7] = np.nan
    srv.submit(s, bad)
    for k in (6, 7):
        srv.submit(s, np.ascontiguousarray(x[k]))
    srv.drain()
    assert s.sync() == fcx.FCX_E_NONFINITE
    assert s.counts() == (7, 1)
    ref = oracle.network(x[[3, 4, 6, 7]].astype(np.float64), c)
    compare_network(s, ref, c, ALL, label="served after rejection")
    fcx.check(s.close())
    fcx.check(srv.destroy())


def test_read_waits_for_queued_trials(fcx):
    """Reads issued right after submissions (no drain) see every trial
    submitted before them: K and the networks are those of the whole
    submitted window, against the oracle; a read of a held server releases
    the hold, and a drain while held is refused."""
    c = synth.base_config(n_nodes=300, n_samples=500, window_trials=6, n_fft=512, f_lo_hz=8, f_hi_hz=30,
                          metrics=synth.ALL8)
    x = synth.c4_trials(c, 21, 17).astype(np.float32)
    srv = fcx.Server(1 << 36)
    st, s = srv.open(c)
    fcx.check(st)
    done = 0
    for burst in (3, 9, 5):
        fcx.check(srv.hold(burst == 9))     # the 9 are queued while held: the read releases the hold
        for k in range(done, done + burst):
            srv.submit(s, np.ascontiguousarray(x[k]))
        done += burst
        if burst == 9:
            assert fcx.lib.fcx_server_drain(srv.h) == fcx.FCX_E_BUSY   # held with trials pending
        W = c["window_trials"]
        ref = oracle.network(x[max(0, done - W):done].astype(np.float64), c)
        compare_network(s, ref, c, ALL, label=f"read after {done} submitted")
    fcx.check(s.close())
    fcx.check(srv.destroy())


def test_full_serving_mix_against_oracle(fcx):
    """The serving mix at its full shape (64 sessions, N in {60, 128, 306,
    1000, 2000}, W ~ U{10..100}, seeded metric subsets): every session's
    window filled and slid through the server (all trials queued while the
    server is held, so they are coalesced in groups of 8), then checked
    against the FP64 oracle: the largest sessions on sampled rows against
    sampled columns, a few small ones in full."""
    sess = synth.c4_sessions(4)
    pool = 6                                   # distinct trials per session, reused in order
    xs = [np.ascontiguousarray(synth.c4_trials(c, sd, pool), dtype=np.float32) for c, sd in sess]
    srv = fcx.Server(int(sum(fcx.server_footprint_bytes(c) for c, _ in sess) * 1.05))
    served = []
    for c, _ in sess:
        st, h = srv.open(c)
        fcx.check(st, "open")
        served.append(h)
    # W + 3 trials per session: the window fills and slides past its first trials
    T = [c["window_trials"] + 3 for c, _ in sess]
    fcx.check(srv.hold(True))
    for r in range(max(T)):
        for k, h in enumerate(served):
            if r < T[k]:
                srv.submit(h, xs[k][r % pool])
    fcx.check(srv.hold(False))
    srv.drain()
    ticks, trials, group, busy = srv.counts()
    log(f"full serving mix: {trials} trials in {ticks} ticks, largest group {group}")
    assert trials == sum(T) and group == 8
    Ns = [c["n_nodes"] for c, _ in sess]
    big = sorted(range(len(sess)), key=lambda k: -Ns[k])[:2]
    small = sorted(range(len(sess)), key=lambda k: Ns[k])[:3]
    rng = np.random.default_rng(11)
    for k in big + small:
        c = sess[k][0]
        N, W = c["n_nodes"], c["window_trials"]
        names = [m for m in ALL if c["metrics"] & synth.METRIC_BITS[m]]
        window = [r % pool for r in range(T[k] - W, T[k])]
        if N > 500:
            rows = [0, 1, N // 2, N - 2]
            cols = sorted(set(rng.choice(N, 64, replace=False).tolist()) | {2, N - 1})
            pi, pj = oracle.row_pairs(rows, N, cols)
            nodes = np.unique(np.concatenate([pi, pj]))
            local = np.full(N, -1, dtype=np.int64)
            local[nodes] = np.arange(nodes.size)
            sub = xs[k][window][:, nodes, :].astype(np.float64)
            ref = oracle.network(sub, dict(c, n_nodes=int(nodes.size)), local[pi], local[pj])
            compare_network(served[k], ref, c, names, idx=oracle.packed_index(pi, pj, N),
                            label=f"served N={N} W={W} (sampled)")
        else:
            ref = oracle.network(xs[k][window].astype(np.float64), c)
            compare_network(served[k], ref, c, names, label=f"served N={N} W={W}")
    for h in served:
        fcx.check(h.close())
    fcx.check(srv.destroy())
