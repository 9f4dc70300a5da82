"""The large multitaper workload at full size: 10000 nodes (50M pairs), DPSS
NW=2 with 3 tapers, 4-40 Hz (37 bins), sliding window of 200 trials x 1000
samples, all 8 metrics (~91 GB of device state).  Sampled rows against
sampled columns are checked against the FP64 oracle after the window has
slid past its first trials."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare_network, log

pytestmark = pytest.mark.gpu

ALL = ["coh", "imcoh", "plv", "pli", "wpli", "uspli", "dswpli", "cor"]


def test_large_multitaper_full_size():
    import torch
    import paper_2303_03279_amd as fcx
    torch.cuda.set_device(0)
    pool = 32
    x, cfg = synth.c5_multitaper(n_trials=pool)
    N, M, W = cfg["n_nodes"], cfg["n_samples"], cfg["window_trials"]
    pushes = W + 9
    order = [k % pool for k in range(pushes)]
    log(f"large multitaper: N={N} W={W} L=3 B=37, {pushes} pushes, footprint "
        f"{fcx.footprint_bytes(cfg) / 1e9:.1f} GB")
    xd = torch.from_numpy(x).cuda()
    torch.cuda.synchronize()
    s = fcx.Session(cfg)
    for k in order:
        fcx.check(s.push_device(xd[k].data_ptr(), M), "push")
    fcx.check(s.sync(), "sync")
    del xd
    rng = np.random.default_rng(55)
    rows = [0, 1, 4999, 9998]
    cols = sorted(set(rng.choice(N, 96, replace=False).tolist()) | {2, 5000, 9999})
    pi, pj = oracle.row_pairs(rows, N, cols)
    nodes = np.unique(np.concatenate([pi, pj]))
    local = np.full(N, -1, dtype=np.int64)
    local[nodes] = np.arange(nodes.size)
    sub = x[:, nodes, :][order[pushes - W:]].astype(np.float64)
    ref = oracle.network(sub, dict(cfg, n_nodes=int(nodes.size)), local[pi], local[pj])
    compare_network(s, ref, cfg, ALL, idx=oracle.packed_index(pi, pj, N), label="large multitaper")
    s.close()
