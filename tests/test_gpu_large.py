"""The large multitaper workload at full size: 10000 nodes (50M pairs), DPSS
NW=2 with 3 tapers, 4-40 Hz (37 bins), sliding window of 200 trials x 1000
samples, all 8 metrics (~91 GB of device state).  Sampled rows against
sampled columns are checked against the FP64 oracle after the window has
slid past its first trials, and for the whole window in one batch pass with
the BF16x3 Gram."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare_network, log

pytestmark = pytest.mark.gpu

ALL = ["coh", "imcoh", "plv", "pli", "wpli", "uspli", "dswpli", "cor"]


POOL = 32   # distinct trials generated (the window reuses them in order)


@pytest.fixture(scope="module")
def c5():
    return synth.c5_multitaper(n_trials=POOL)


def _sampled_pairs(N):
    rng = np.random.default_rng(55)
    rows = [0, 1, 4999, 9998]
    cols = sorted(set(rng.choice(N, 96, replace=False).tolist()) | {2, 5000, 9999})
    return oracle.row_pairs(rows, N, cols)


def _oracle_sampled(x, trials, cfg, pi, pj):
    N = cfg["n_nodes"]
    nodes = np.unique(np.concatenate([pi, pj]))
    local = np.full(N, -1, dtype=np.int64)
    local[nodes] = np.arange(nodes.size)
    sub = x[:, nodes, :][trials].astype(np.float64)
    return oracle.network(sub, dict(cfg, n_nodes=int(nodes.size)), local[pi], local[pj])


def test_large_multitaper_full_size(c5):
    import torch
    import paper_2303_03279_amd as fcx
    torch.cuda.set_device(0)
    pool = POOL
    x, cfg = c5
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
    pi, pj = _sampled_pairs(N)
    ref = _oracle_sampled(x, order[pushes - W:], cfg, pi, pj)
    compare_network(s, ref, cfg, ALL, idx=oracle.packed_index(pi, pj, N), label="large multitaper")
    s.close()


def test_large_multitaper_batch_bf16x3(c5):
    """The same workload's whole window of 200 trials in one batch pass with
    the split BF16x3 Gram (the workload's Gram precision), sampled rows
    against the FP64 oracle at the 1e-5 bound."""
    import torch
    import paper_2303_03279_amd as fcx
    torch.cuda.set_device(0)
    x, cfg = c5
    N, M, W = cfg["n_nodes"], cfg["n_samples"], cfg["window_trials"]
    assert cfg["gram"] == "bf16x3"
    trials = [k % POOL for k in range(W)]
    xd = torch.from_numpy(x).cuda()[torch.tensor(trials)].contiguous()   # [W][N][M] on the device
    torch.cuda.synchronize()
    s = fcx.Session(cfg)
    fcx.check(s.push_batch_device(xd.data_ptr(), W, N * M, M), "push_batch")
    fcx.check(s.sync(), "sync")
    del xd
    torch.cuda.empty_cache()
    pi, pj = _sampled_pairs(N)
    ref = _oracle_sampled(x, trials, cfg, pi, pj)
    compare_network(s, ref, cfg, ALL, idx=oracle.packed_index(pi, pj, N), label="large multitaper batch bf16x3")
    s.close()
