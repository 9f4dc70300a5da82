"""Python binding of the fcx C ABI (include/fcx.h): argument marshalling only.

Every step of the connectivity path runs in the HIP library libfcx.so built
in this directory; this module only loads it, declares the C signatures and
converts arguments.  There is no fallback: if the library is missing the
import fails.

torch, when present, is imported first so that the library binds to the same
HIP runtime that torch already loaded (torch tensors then serve as device
buffers and torch streams as HIP streams).
"""
from __future__ import annotations

import ctypes
import os

try:  # share torch's HIP runtime if torch is around
    import torch  # noqa: F401
except Exception:  # pragma: no cover - the library does not need torch
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfcx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2303_03279_amd.build` "
                      "(hipcc, gfx950); there is no fallback implementation")

lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants
FCX_OK, FCX_E_INVAL, FCX_E_NOMEM, FCX_E_DEVICE, FCX_E_NOTREADY, FCX_E_BUSY, FCX_E_CLOSED, \
    FCX_E_NONFINITE = range(8)
FCX_COH, FCX_IMCOH, FCX_PLV, FCX_PLI, FCX_WPLI, FCX_USPLI, FCX_DSWPLI, FCX_COR, FCX_XCOR = (
    1, 2, 4, 8, 16, 32, 64, 128, 256)
FCX_TAPER_HANN, FCX_TAPER_DPSS = 0, 1
FCX_GRAM_FP32, FCX_GRAM_BF16, FCX_GRAM_BF16X3 = 0, 1, 2
FCX_ELEM_F32, FCX_ELEM_F64 = 0, 1
(FCX_K_SPECTRA, FCX_K_PSD, FCX_K_PAIR_UPDATE, FCX_K_COR, FCX_K_PAIR_BATCH, FCX_K_ZNORM, FCX_K_XCOR,
 FCX_K_COUNT) = range(8)

METRIC_BITS = dict(coh=FCX_COH, imcoh=FCX_IMCOH, plv=FCX_PLV, pli=FCX_PLI, wpli=FCX_WPLI,
                   uspli=FCX_USPLI, dswpli=FCX_DSWPLI, cor=FCX_COR, xcor=FCX_XCOR)
BROADBAND = ("cor", "xcor")


class fcx_config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("n_nodes", ctypes.c_int32),
        ("n_samples", ctypes.c_int32),
        ("window_trials", ctypes.c_int32),
        ("n_fft", ctypes.c_int32),
        ("fs_hz", ctypes.c_double),
        ("f_lo_hz", ctypes.c_double),
        ("f_hi_hz", ctypes.c_double),
        ("taper", ctypes.c_int32),
        ("dpss_k", ctypes.c_int32),
        ("dpss_nw", ctypes.c_double),
        ("metrics", ctypes.c_uint32),
        ("gram_precision", ctypes.c_int32),
        ("elem", ctypes.c_int32),
        ("xcor_max_lag", ctypes.c_int32),
    ]


class fcx_select_info(ctypes.Structure):
    _fields_ = [
        ("max_abs", ctypes.c_float),
        ("threshold", ctypes.c_float),
        ("k", ctypes.c_int64),
        ("n_finite", ctypes.c_int64),
        ("n_selected", ctypes.c_int64),
    ]


class fcx_stream_config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("n_channels", ctypes.c_int32),
        ("block_len", ctypes.c_int32),
        ("n_taps", ctypes.c_int32),
        ("taps", ctypes.c_void_p),
        ("trigger_threshold", ctypes.c_float),
        ("pre_samples", ctypes.c_int32),
        ("post_samples", ctypes.c_int32),
    ]


FCX_FIR_LOWPASS, FCX_FIR_HIGHPASS, FCX_FIR_BANDPASS = 0, 1, 2


GRAMS = {"fp32": FCX_GRAM_FP32, "bf16": FCX_GRAM_BF16, "bf16x3": FCX_GRAM_BF16X3}


class fcx_hilbert_config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("n_nodes", ctypes.c_int32),
        ("n_samples", ctypes.c_int32),
        ("n_taps", ctypes.c_int32),
        ("taps", ctypes.c_void_p),
        ("win_len", ctypes.c_int32),
        ("win_hop", ctypes.c_int32),
        ("metrics", ctypes.c_uint32),
        ("gram_precision", ctypes.c_int32),
    ]

P = ctypes.c_void_p
I32, I64, U32, U64, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
PI32, PI64, PD, PU64 = (ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64))
PCFG = ctypes.POINTER(fcx_config)
PP = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "fcx_config_init": (None, [PCFG]),
    "fcx_footprint_bytes": (I64, [PCFG]),
    "fcx_server_footprint_bytes": (I64, [PCFG]),
    "fcx_pair_update_bytes": (I64, [PCFG]),
    "fcx_band_bins": (I32, [PCFG, PI32, PI32]),
    "fcx_open": (ctypes.c_int, [PCFG, P, PP]),
    "fcx_push_trial": (ctypes.c_int, [P, P, I64, ctypes.c_int]),
    "fcx_push_batch": (ctypes.c_int, [P, P, I64, I64, I64, ctypes.c_int]),
    "fcx_read_network": (ctypes.c_int, [P, U32, P, I64, ctypes.c_int, ctypes.c_int, PI32]),
    "fcx_sync": (ctypes.c_int, [P]),
    "fcx_resync": (ctypes.c_int, [P]),
    "fcx_close": (ctypes.c_int, [P]),
    "fcx_session_stream": (ctypes.c_int, [P, PP]),
    "fcx_session_counts": (ctypes.c_int, [P, PI64, PI64]),
    "fcx_set_timing": (ctypes.c_int, [P, ctypes.c_int]),
    "fcx_kernel_time": (ctypes.c_int, [P, ctypes.c_int, PI64, PD]),
    "fcx_dpss": (ctypes.c_int, [I32, D, I32, P, P]),
    "fcx_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "fcx_probe_copy": (ctypes.c_int, [P, P, I64, P]),
    "fcx_probe_rmw": (ctypes.c_int, [P, I64, P]),
    "fcx_probe_mfma": (ctypes.c_int, [I32, I32, P, ctypes.POINTER(ctypes.c_double), P]),
    "fcx_network_select": (ctypes.c_int, [I32, P, D, P, P, P, P, ctypes.POINTER(fcx_select_info), P]),
    "fcx_network_select_noalloc": (ctypes.c_int, [I32, P, D, P, P, P, P, ctypes.POINTER(fcx_select_info), P]),
    "fcx_fir_design": (ctypes.c_int, [I32, D, D, D, D, I32, P, I32, PI32]),
    "fcx_stream_open": (ctypes.c_int, [ctypes.POINTER(fcx_stream_config), P, PP]),
    "fcx_stream_push": (ctypes.c_int, [P, P, I64, P, P, P, I32, PI32, PI32]),
    "fcx_stream_close": (ctypes.c_int, [P]),
    "fcx_hilbert_open": (ctypes.c_int, [ctypes.POINTER(fcx_hilbert_config), P, PP]),
    "fcx_hilbert_info": (ctypes.c_int, [P, PI32, PI32]),
    "fcx_hilbert_run": (ctypes.c_int, [P, P, I64, P, P]),
    "fcx_hilbert_close": (ctypes.c_int, [P]),
    "fcx_server_create": (ctypes.c_int, [I64, PP]),
    "fcx_server_open": (ctypes.c_int, [P, PCFG, PP]),
    "fcx_server_submit": (ctypes.c_int, [P, P, P, I64, PU64]),
    "fcx_server_poll": (ctypes.c_int, [P, U64, ctypes.POINTER(ctypes.c_int), PD]),
    "fcx_server_drain": (ctypes.c_int, [P]),
    "fcx_server_usage": (ctypes.c_int, [P, PI64, PI64, PI32]),
    "fcx_server_counts": (ctypes.c_int, [P, PI64, PI64, PI64, PD]),
    "fcx_server_hold": (ctypes.c_int, [P, I32]),
    "fcx_server_close_session": (ctypes.c_int, [P, P]),
    "fcx_server_destroy": (ctypes.c_int, [P]),
}

for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn

EXPORTED = tuple(_SIGS)


class FcxError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {lib.fcx_status_str(status).decode()} ({status})")


def check(status: int, where: str = "fcx") -> int:
    if status != FCX_OK:
        raise FcxError(status, where)
    return status


def network_select(n_nodes: int, w_ptr: int, fraction: float, w_norm_ptr: int = 0, selected_ptr: int = 0,
                   degree_ptr: int = 0, strength_ptr: int = 0, stream: int = 0):
    """fcx_network_select on device buffers (pointers as ints, 0 = not
    wanted).  Returns (status, info dict)."""
    info = fcx_select_info()
    st = lib.fcx_network_select(int(n_nodes), w_ptr, float(fraction), w_norm_ptr or None, selected_ptr or None,
                                degree_ptr or None, strength_ptr or None, ctypes.byref(info), stream or None)
    return st, dict(max_abs=info.max_abs, threshold=info.threshold, k=info.k, n_finite=info.n_finite,
                    n_selected=info.n_selected)


def network_select_noalloc(n_nodes: int, w_ptr: int, fraction: float, w_norm_ptr: int = 0, selected_ptr: int = 0,
                           degree_ptr: int = 0, strength_ptr: int = 0, stream: int = 0, want_info: bool = True):
    """fcx_network_select_noalloc on device buffers.  With want_info False
    the call only enqueues (info None).  Returns (status, info dict or None)."""
    info = fcx_select_info()
    st = lib.fcx_network_select_noalloc(int(n_nodes), w_ptr, float(fraction), w_norm_ptr or None,
                                        selected_ptr or None, degree_ptr or None, strength_ptr or None,
                                        ctypes.byref(info) if want_info else None, stream or None)
    if not want_info:
        return st, None
    return st, dict(max_abs=info.max_abs, threshold=info.threshold, k=info.k, n_finite=info.n_finite,
                    n_selected=info.n_selected)


def fir_design(kind: int, fs: float, f1: float, f2: float = 0.0, transition_hz: float = 0.0, n_taps: int = 0):
    """fcx_fir_design: the taps as a float64 array."""
    import numpy as np
    n = ctypes.c_int32()
    check(lib.fcx_fir_design(kind, fs, f1, f2, transition_hz, n_taps, None, 0, ctypes.byref(n)), "fir_design")
    taps = np.empty(n.value)
    check(lib.fcx_fir_design(kind, fs, f1, f2, transition_hz, n_taps, taps.ctypes.data, n.value, ctypes.byref(n)),
          "fir_design")
    return taps


class Stream:
    """Stream front end (fcx_stream_*): block filtering and trial cutting on
    device buffers (pointers as ints)."""

    def __init__(self, n_channels: int, block_len: int, taps, threshold: float, pre: int, post: int,
                 stream: int = 0):
        import numpy as np
        self.taps = np.ascontiguousarray(taps, dtype=np.float64)
        c = fcx_stream_config()
        c.struct_size = ctypes.sizeof(fcx_stream_config)
        c.n_channels, c.block_len, c.n_taps = int(n_channels), int(block_len), int(self.taps.size)
        c.taps = self.taps.ctypes.data
        c.trigger_threshold = float(threshold)
        c.pre_samples, c.post_samples = int(pre), int(post)
        self.h = ctypes.c_void_p()
        check(lib.fcx_stream_open(ctypes.byref(c), stream or None, ctypes.byref(self.h)), "stream_open")
        self.C, self.block_len, self.len = n_channels, block_len, pre + post
        self.delay = (self.taps.size - 1) // 2

    def push(self, x_ptr: int, ld: int, trig_ptr: int, y_ptr: int = 0, trials_ptr: int = 0, cap: int = 0):
        """Returns (status, n_trials, n_dropped)."""
        n, d = ctypes.c_int32(), ctypes.c_int32()
        st = lib.fcx_stream_push(self.h, x_ptr, ld, trig_ptr, y_ptr or None, trials_ptr or None, cap,
                                 ctypes.byref(n), ctypes.byref(d))
        return st, n.value, d.value

    def close(self) -> int:
        return lib.fcx_stream_close(self.h)


class Hilbert:
    """Time-resolved analytic-signal connectivity (fcx_hilbert_*) on device
    buffers (pointers as ints)."""

    def __init__(self, n_nodes: int, n_samples: int, taps, win_len: int = 0, win_hop: int = 0,
                 metrics: int = 0x7F, gram: str = "fp32", stream: int = 0):
        import numpy as np
        self.taps = np.ascontiguousarray(taps, dtype=np.float64)
        c = fcx_hilbert_config()
        c.struct_size = ctypes.sizeof(fcx_hilbert_config)
        c.n_nodes, c.n_samples, c.n_taps = int(n_nodes), int(n_samples), int(self.taps.size)
        c.taps = self.taps.ctypes.data
        c.win_len, c.win_hop, c.metrics = int(win_len), int(win_hop), int(metrics)
        c.gram_precision = GRAMS[gram]
        self.h = ctypes.c_void_p()
        check(lib.fcx_hilbert_open(ctypes.byref(c), stream or None, ctypes.byref(self.h)), "hilbert_open")
        nw, F = ctypes.c_int32(), ctypes.c_int32()
        check(lib.fcx_hilbert_info(self.h, ctypes.byref(nw), ctypes.byref(F)), "hilbert_info")
        self.N, self.M, self.n_windows, self.fft_len = n_nodes, n_samples, nw.value, F.value
        self.P = n_nodes * (n_nodes - 1) // 2

    def run(self, x_ptr: int, ld: int, out_ptr: int, z_ptr: int = 0) -> int:
        return lib.fcx_hilbert_run(self.h, x_ptr, ld, out_ptr, z_ptr or None)

    def close(self) -> int:
        return lib.fcx_hilbert_close(self.h)


def make_config(cfg: dict) -> fcx_config:
    """fcx_config from a plain dict (keys as in the C struct; taper 'hann'/'dpss',
    gram 'fp32'/'bf16'/'bf16x3', elem 'f32'/'f64')."""
    c = fcx_config()
    lib.fcx_config_init(ctypes.byref(c))
    c.n_nodes = int(cfg["n_nodes"])
    c.n_samples = int(cfg["n_samples"])
    c.window_trials = int(cfg["window_trials"])
    c.n_fft = int(cfg["n_fft"])
    c.fs_hz = float(cfg["fs_hz"])
    c.f_lo_hz = float(cfg["f_lo_hz"])
    c.f_hi_hz = float(cfg["f_hi_hz"])
    c.taper = {"hann": FCX_TAPER_HANN, "dpss": FCX_TAPER_DPSS}[cfg.get("taper", "hann")]
    c.dpss_nw = float(cfg.get("dpss_nw", 0.0))
    c.dpss_k = int(cfg.get("dpss_k", 0))
    c.metrics = int(cfg.get("metrics", 255))
    c.gram_precision = GRAMS[cfg.get("gram", "fp32")]
    c.elem = {"f32": FCX_ELEM_F32, "f64": FCX_ELEM_F64}[cfg.get("elem", "f32")]
    c.xcor_max_lag = int(cfg.get("xcor_max_lag", 0))
    return c


def footprint_bytes(cfg: dict) -> int:
    c = make_config(cfg)
    return int(lib.fcx_footprint_bytes(ctypes.byref(c)))


def server_footprint_bytes(cfg: dict) -> int:
    c = make_config(cfg)
    return int(lib.fcx_server_footprint_bytes(ctypes.byref(c)))


def pair_update_bytes(cfg: dict) -> int:
    c = make_config(cfg)
    return int(lib.fcx_pair_update_bytes(ctypes.byref(c)))


def band_bins(cfg: dict):
    c = make_config(cfg)
    lo, hi = ctypes.c_int32(), ctypes.c_int32()
    n = lib.fcx_band_bins(ctypes.byref(c), ctypes.byref(lo), ctypes.byref(hi))
    return int(n), int(lo.value), int(hi.value)


def dpss(M: int, NW: float, K: int):
    import numpy as np
    tap = np.empty((K, M))
    rat = np.empty(K)
    check(lib.fcx_dpss(M, NW, K, tap.ctypes.data, rat.ctypes.data), "fcx_dpss")
    return tap, rat


class Session:
    """Owning wrapper of an fcx_session handle (marshalling only)."""

    def __init__(self, cfg: dict, stream=None):
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        h = ctypes.c_void_p()
        check(lib.fcx_open(ctypes.byref(self._c), stream, ctypes.byref(h)), "fcx_open")
        self.h = h
        self.N = int(cfg["n_nodes"])
        self.P = self.N * (self.N - 1) // 2
        self.B, self.klo, self.khi = band_bins(cfg)
        self.f64 = cfg.get("elem", "f32") == "f64"

    # -- pushes --------------------------------------------------------------
    def push_host(self, x) -> int:
        """x: numpy array [N][M] of the session's element type."""
        return lib.fcx_push_trial(self.h, x.ctypes.data, x.strides[0] // x.itemsize, 0)

    def push_device(self, ptr: int, ld: int) -> int:
        return lib.fcx_push_trial(self.h, ptr, ld, 1)

    def push_batch_device(self, ptr: int, n_trials: int, trial_stride: int, ld: int) -> int:
        return lib.fcx_push_batch(self.h, ptr, n_trials, trial_stride, ld, 1)

    def push_batch_host(self, x) -> int:
        """x: numpy array [K][N][M] of the session's element type (rows and
        trials may be strided, samples contiguous)."""
        if x.ndim != 3 or x.strides[2] != x.itemsize:
            raise ValueError("push_batch_host takes a [K][N][M] array with contiguous samples")
        return lib.fcx_push_batch(self.h, x.ctypes.data, x.shape[0], x.strides[0] // x.itemsize,
                                  x.strides[1] // x.itemsize, 0)

    # -- reads ---------------------------------------------------------------
    def read(self, metric: str, per_bin: bool = False):
        import numpy as np
        bit = METRIC_BITS[metric]
        n = self.P * (self.B if (per_bin and metric not in BROADBAND) else 1)
        out = np.empty(n, dtype=np.float64 if self.f64 else np.float32)
        k = ctypes.c_int32()
        st = lib.fcx_read_network(self.h, bit, out.ctypes.data, n, 0, int(per_bin), ctypes.byref(k))
        if per_bin and metric not in BROADBAND:
            out = out.reshape(self.B, self.P)
        return st, out, int(k.value)

    def read_device(self, metric: str, ptr: int, n: int, per_bin: bool = False) -> int:
        k = ctypes.c_int32()
        return lib.fcx_read_network(self.h, METRIC_BITS[metric], ptr, n, 1, int(per_bin), ctypes.byref(k))

    def sync(self) -> int:
        return lib.fcx_sync(self.h)

    def resync(self) -> int:
        return lib.fcx_resync(self.h)

    def counts(self):
        a, r = ctypes.c_int64(), ctypes.c_int64()
        check(lib.fcx_session_counts(self.h, ctypes.byref(a), ctypes.byref(r)), "fcx_session_counts")
        return int(a.value), int(r.value)

    def stream(self) -> int:
        p = ctypes.c_void_p()
        check(lib.fcx_session_stream(self.h, ctypes.byref(p)), "fcx_session_stream")
        return int(p.value or 0)

    def set_timing(self, on: bool):
        check(lib.fcx_set_timing(self.h, int(on)), "fcx_set_timing")

    def kernel_time(self, kernel: int):
        n, ms = ctypes.c_int64(), ctypes.c_double()
        check(lib.fcx_kernel_time(self.h, kernel, ctypes.byref(n), ctypes.byref(ms)), "fcx_kernel_time")
        return int(n.value), float(ms.value)

    def close(self) -> int:
        if self.h is None:
            return FCX_OK
        st = lib.fcx_close(self.h)
        self.h = None
        return st

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                lib.fcx_close(self.h)
        except Exception:
            pass


class Server:
    """Owning wrapper of an fcx_server handle (marshalling only)."""

    def __init__(self, hbm_budget_bytes: int):
        h = ctypes.c_void_p()
        check(lib.fcx_server_create(int(hbm_budget_bytes), ctypes.byref(h)), "fcx_server_create")
        self.h = h

    def open(self, cfg: dict):
        """Returns (status, ServedSession or None)."""
        c = make_config(cfg)
        h = ctypes.c_void_p()
        st = lib.fcx_server_open(self.h, ctypes.byref(c), ctypes.byref(h))
        if st != FCX_OK:
            return st, None
        return st, ServedSession(self, cfg, h)

    def submit(self, sess, x) -> int:
        t = ctypes.c_uint64()
        check(lib.fcx_server_submit(self.h, sess.h, x.ctypes.data, x.strides[0] // x.itemsize,
                                    ctypes.byref(t)), "fcx_server_submit")
        return int(t.value)

    def poll(self, ticket: int):
        done, lat = ctypes.c_int(), ctypes.c_double()
        check(lib.fcx_server_poll(self.h, ticket, ctypes.byref(done), ctypes.byref(lat)), "fcx_server_poll")
        return bool(done.value), float(lat.value)

    def drain(self):
        check(lib.fcx_server_drain(self.h), "fcx_server_drain")

    def usage(self):
        u, l, n = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        check(lib.fcx_server_usage(self.h, ctypes.byref(u), ctypes.byref(l), ctypes.byref(n)), "fcx_server_usage")
        return int(u.value), int(l.value), int(n.value)

    def hold(self, on: bool) -> int:
        return lib.fcx_server_hold(self.h, 1 if on else 0)

    def counts(self):
        """(ticks run, trials applied, largest coalesced group, device ms of the ticks)."""
        t, n, g, ms = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        check(lib.fcx_server_counts(self.h, ctypes.byref(t), ctypes.byref(n), ctypes.byref(g), ctypes.byref(ms)),
              "server_counts")
        return t.value, n.value, g.value, ms.value

    def close_session(self, sess) -> int:
        st = lib.fcx_server_close_session(self.h, sess.h)
        sess.h = None
        return st

    def destroy(self) -> int:
        if self.h is None:
            return FCX_OK
        st = lib.fcx_server_destroy(self.h)
        self.h = None
        return st


class ServedSession(Session):
    """A session owned by a server: trials go through Server.submit, reads are
    the same as for a plain session."""

    def __init__(self, server, cfg, h):  # noqa: D401 - no fcx_open here
        self.cfg = dict(cfg)
        self.h = h
        self.server = server
        self.N = int(cfg["n_nodes"])
        self.P = self.N * (self.N - 1) // 2
        self.B, self.klo, self.khi = band_bins(cfg)
        self.f64 = False

    def close(self) -> int:
        if self.h is None:
            return FCX_OK
        return self.server.close_session(self)

    def __del__(self):
        pass
