"""The allocation-free network selection (fcx_network_select_noalloc)
against the allocating entry point (fcx_network_select) on the same
networks, bit for bit: two calls in a row, the second on a smaller network
(the shared device array keeps the first call's contents), one of them only
enqueued (no info, no wait), and the size limit."""
import numpy as np
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fcx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2303_03279_amd as m
    return m


def _network(N, seed):
    rng = np.random.default_rng(seed)
    P = N * (N - 1) // 2
    w = rng.standard_normal(P).astype(np.float32)
    w[rng.integers(0, P, size=P // 50)] = np.float32(0.5)      # ties at one weight
    w[rng.integers(0, P, size=3)] = np.nan                      # non-finite edges are never selected
    return w


def _select(fcx, fn, w, N, fraction, want_info=True):
    import torch
    P = N * (N - 1) // 2
    wd = torch.from_numpy(w).cuda()
    w_norm = torch.full((P,), 7.0, dtype=torch.float32, device="cuda")
    sel = torch.full((P,), 9, dtype=torch.uint8, device="cuda")
    deg = torch.full((N,), -1, dtype=torch.int32, device="cuda")
    stren = torch.full((N,), -1.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    if fn == "noalloc":
        st, info = fcx.network_select_noalloc(N, wd.data_ptr(), fraction, w_norm.data_ptr(), sel.data_ptr(),
                                              deg.data_ptr(), stren.data_ptr(), want_info=want_info)
    else:
        st, info = fcx.network_select(N, wd.data_ptr(), fraction, w_norm.data_ptr(), sel.data_ptr(),
                                      deg.data_ptr(), stren.data_ptr())
    fcx.check(st, fn)
    torch.cuda.synchronize()
    return info, w_norm.cpu().numpy(), sel.cpu().numpy(), deg.cpu().numpy(), stren.cpu().numpy()


def _same(a, b, label):
    ia, ib = a[0], b[0]
    if ia is not None and ib is not None:
        for k in ("k", "n_finite", "n_selected"):
            assert ia[k] == ib[k], (label, k)
        for k in ("max_abs", "threshold"):
            assert np.float32(ia[k]) == np.float32(ib[k]), (label, k)
    for x, y, name in zip(a[1:], b[1:], ("w_norm", "selected", "degree", "strength")):
        assert np.array_equal(x, y, equal_nan=True), (label, name)


@pytest.mark.parametrize("second_info", [True, False])
def test_noalloc_equals_select(fcx, second_info):
    for N, frac, seed in ((3000, 0.05, 1), (700, 0.10, 2)):
        log(f"noalloc: N={N} f={frac}")
        w = _network(N, seed)
        ref = _select(fcx, "select", w, N, frac)
        got = _select(fcx, "noalloc", w, N, frac, want_info=second_info or N == 3000)
        _same(got, ref, f"N={N}")
        assert ref[0]["n_selected"] >= ref[0]["k"] > 0


def test_noalloc_rejects_oversize(fcx):
    import torch
    w = torch.zeros(16, dtype=torch.float32, device="cuda")
    st, _ = fcx.network_select_noalloc(65537, w.data_ptr(), 0.05)
    assert st == fcx.FCX_E_INVAL
    st, _ = fcx.network_select_noalloc(1, w.data_ptr(), 0.05)
    assert st == fcx.FCX_E_INVAL


def test_noalloc_under_graph_capture(fcx):
    """The enqueue-only form (no info) captured in a HIP graph through
    torch.cuda.graph and replayed three times, the network rewritten eagerly
    in the same buffer before each replay and the allocating call run eagerly
    after it: every replay's outputs equal that call's, bit for bit."""
    import torch
    N, frac = 900, 0.05
    P = N * (N - 1) // 2
    w = torch.from_numpy(_network(N, 11)).cuda()
    w_norm = torch.empty(P, dtype=torch.float32, device="cuda")
    sel = torch.empty(P, dtype=torch.uint8, device="cuda")
    deg = torch.empty(N, dtype=torch.int32, device="cuda")
    stren = torch.empty(N, dtype=torch.float32, device="cuda")
    args = (N, w.data_ptr(), frac, w_norm.data_ptr(), sel.data_ptr(), deg.data_ptr(), stren.data_ptr())
    # eager warm-up on a side stream: the first call on the device looks up the array
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fcx.check(fcx.network_select_noalloc(*args, stream=side.cuda_stream, want_info=False)[0], "warm-up")
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        st, _ = fcx.network_select_noalloc(*args, stream=torch.cuda.current_stream().cuda_stream, want_info=False)
    fcx.check(st, "capture")
    torch.cuda.synchronize()
    for rep in range(3):
        log(f"graph replay {rep}")
        data = _network(N, 20 + rep) * np.float32(rep + 1)
        w.copy_(torch.from_numpy(data))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (None, w_norm.cpu().numpy(), sel.cpu().numpy(), deg.cpu().numpy(), stren.cpu().numpy())
        ref = _select(fcx, "select", data, N, frac)
        _same(got, ref, f"replay {rep}")
        assert int(got[2].sum()) == ref[0]["n_selected"] > 0
    del g
