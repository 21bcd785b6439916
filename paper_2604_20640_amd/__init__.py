"""qc: an FX-correlator hot path for AMD MI355X (gfx950), after arXiv 2604.20640.

A thin ctypes binding over ``libqc.so`` (C ABI in ``include/qc.h``).  The
functions here only marshal arguments: every step runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.  If the
library is missing this module raises on first use; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "QCError", "lib", "pfb_channelize", "xcorrelate", "xcorrelate_noalloc", "xcorrelate_chan",
    "pfb_channelize_ex", "xcorrelate_ex", "design_taps", "SAMPLE", "WINDOW", "image_grid", "image_invert",
    "image_clean", "image_dirty_and_psf", "ingest_run", "IngestConfig", "IngestStats", "mad_flag",
    "apply_delay_phase", "n_base", "PREC", "timing_enable", "timing_read", "KERNELS", "Stream",
    "solve_delay_phase", "Plan", "cnn_param_count", "cnn_normalize", "cnn_forward", "cnn_grad", "cnn_adam",
    "cnn_train_step", "cnn_flag", "channelize_variant", "cnn_variant", "measure_peak",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqc.so")

PREC = {"f32": 0, "f16": 1, "bf16": 2, "fp8": 3}
SAMPLE = {"i8": 0, "i16": 1, "ci8": 2, "ci16": 3}
WINDOW = {"hann": 0, "kaiser": 1, "rect": 2}
_PAIR_BYTES = {0: 8, 1: 4, 2: 4, 3: 2}


class QCError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where} failed: status {status} ({detail})")
        self.status = status


class PfbParams(ctypes.Structure):
    _fields_ = [("n_fft", ctypes.c_int32), ("n_taps", ctypes.c_int32),
                ("taps", ctypes.c_void_p), ("keep_nyquist", ctypes.c_int32)]


class IngestConfig(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int32), ("sample", ctypes.c_int32), ("packet_samp", ctypes.c_int64),
                ("batch_packets", ctypes.c_int32), ("queue_max", ctypes.c_int32), ("n_readers", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("pfb", PfbParams), ("spec_per_dump", ctypes.c_int64)]


class IngestStats(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_int64), ("batches", ctypes.c_int64), ("dumps", ctypes.c_int64),
                ("wall_s", ctypes.c_double), ("read_s", ctypes.c_double), ("h2d_s", ctypes.c_double),
                ("compute_s", ctypes.c_double), ("wait_s", ctypes.c_double)]


class ArrayDesc(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int32), ("n_samp", ctypes.c_int64), ("n_fft", ctypes.c_int32),
                ("n_taps", ctypes.c_int32), ("spec_per_dump", ctypes.c_int64)]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SIGS = {
    "qc_pfb_channelize": [_P, _I64, _I32, _I64, ctypes.POINTER(PfbParams), _P, _P, _I32, _P, _P, _P],
    "qc_xcorrelate": [_P, _I64, _I32, _I64, ctypes.POINTER(PfbParams), _P, _P, _I64, _I32, _P, _I32,
                      ctypes.POINTER(_I64), _P],
    "qc_xcorrelate_noalloc": [_P, _I64, _I32, _I64, ctypes.POINTER(PfbParams), _P, _P, _I64, _P, _I32,
                              ctypes.POINTER(_I64), _P],
    "qc_xcorrelate_chan": [_P, _I32, _P, _I32, _I64, _I32, _I64, _P, _I32, _P],
    "qc_pfb_channelize_ex": [_P, _I32, _I64, _I32, _I64, ctypes.POINTER(PfbParams), _P, _P, _I32, _P, _P,
                             _P],
    "qc_xcorrelate_ex": [_P, _I32, _I64, _I32, _I64, ctypes.POINTER(PfbParams), _P, _P, _I64, _I32, _P,
                         _I32, ctypes.POINTER(_I64), _P],
    "qc_pfb_design_taps": [_I32, _I32, _I32, ctypes.c_double, _P, _P],
    "qc_image_grid": [_P, _P, _P, _P, _I64, _I32, ctypes.c_double, _P, _P, _P],
    "qc_ingest_run": [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(IngestConfig), _P, _I64,
                      ctypes.POINTER(IngestStats)],
    "qc_image_invert": [_P, _P, _I32, _P, _P, _P],
    "qc_image_clean": [_P, _P, _I32, ctypes.c_float, ctypes.c_float, _I32, _P, _P, _P, _P],
    "qc_mad_flag": [_P, _I64, _I64, _I32, ctypes.c_float, _I32, _P, _P, _P],
    "qc_apply_delay_phase": [_P, _I64, _I32, _I32, ctypes.c_double, ctypes.c_double,
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _P],
}


def lib() -> ctypes.CDLL:
    """Load libqc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2604_20640_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        L.qc_status_string.restype = ctypes.c_char_p
        L.qc_status_string.argtypes = [ctypes.c_int32]
        L.qc_last_error.restype = ctypes.c_char_p
        L.qc_version.restype = ctypes.c_char_p
        L.qc_stream_create.argtypes = [_I32, _I64, ctypes.POINTER(PfbParams), _I64, _I32,
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.qc_stream_create.restype = ctypes.c_int32
        L.qc_stream_push.argtypes = [_P, _P, _I64, _P, ctypes.POINTER(_I64)]
        L.qc_stream_push.restype = ctypes.c_int32
        L.qc_stream_valid_spectra.argtypes = [_P, ctypes.POINTER(_I64), _I64]
        L.qc_stream_valid_spectra.restype = ctypes.c_int32
        L.qc_stream_wait_copied.argtypes = [_P, _I64]
        L.qc_stream_wait_copied.restype = ctypes.c_int32
        L.qc_stream_sync.argtypes = [_P]
        L.qc_stream_sync.restype = ctypes.c_int32
        L.qc_stream_compute_stream.argtypes = [_P]
        L.qc_stream_compute_stream.restype = ctypes.c_void_p
        L.qc_stream_destroy.argtypes = [_P]
        L.qc_stream_destroy.restype = None
        L.qc_stream_last_error.restype = ctypes.c_char_p
        L.qc_fx_tile_count.argtypes = [_I32, _I32]
        L.qc_fx_tile_count.restype = ctypes.c_int32
        L.qc_fx_set_tile.argtypes = [_I32, _I32, _I32]
        L.qc_fx_set_tile.restype = ctypes.c_int32
        L.qc_fx_get_tile.argtypes = [_I32, _I32]
        L.qc_fx_get_tile.restype = ctypes.c_int32
        L.qc_fx_set_width.argtypes = [_I32, _I32, _I64]
        L.qc_fx_set_width.restype = ctypes.c_int32
        L.qc_fx_get_width.argtypes = [_I32, _I32]
        L.qc_fx_get_width.restype = ctypes.c_int64
        L.qc_fx_autotune.argtypes = [_P, _I64, _I32, _I64, ctypes.POINTER(PfbParams), _I64, _I32, _P,
                                     ctypes.POINTER(ctypes.c_double), _I32, ctypes.POINTER(_I32), _P]
        L.qc_fx_autotune.restype = ctypes.c_int32
        L.qc_solve_delay_phase.argtypes = [_P, _P, _I64, _I32, _I32, ctypes.c_double, ctypes.c_double,
                                           _I32, _I32, _I32, _I32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), _P]
        L.qc_solve_delay_phase.restype = ctypes.c_int32
        PP = ctypes.POINTER(ctypes.c_void_p)
        for name, args in {
            "qc_plan_create": [ctypes.POINTER(ArrayDesc), _I32, ctypes.POINTER(ctypes.c_void_p)],
            "qc_plan_execute": [_P, PP, PP, _P],
            "qc_plan_execute_separate": [_P, PP, PP, _P],
            "qc_plan_check": [_P, _P],
            "qc_plan_set_wait_timeout": [_P, _I64],
            "qc_plan_set_wait_bias": [_P, _I32],
            "qc_plan_capture_graph": [_P, PP, PP, _P],
            "qc_plan_replay": [_P, _P],
            "qc_plan_autotune": [_P, PP, PP, _I32, ctypes.c_char_p, ctypes.POINTER(_I32), _P],
            "qc_plan_info": [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                             ctypes.POINTER(_I64)],
            "qc_plan_set_mode": [_P, _I32],
        }.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        L.qc_plan_destroy.argtypes = [_P]
        L.qc_plan_destroy.restype = None
        _F = ctypes.c_float
        for name, args in {
            "qc_cnn_normalize": [_P, _I64, _I64, _I32, _P, _P],
            "qc_cnn_forward": [_P, _P, _I32, _I32, _I32, _I32, _P, _P],
            "qc_cnn_grad": [_P, _P, _P, _I32, _I32, _I32, _F, _P, _P, _P],
            "qc_cnn_adam": [_P, _P, _P, _P, _I64, _F, _F, _F, _F, _P],
            "qc_cnn_train_step": [_P, _P, _P, _I64, _P, _P, _I32, _I32, _I32, _F, _F, _P, _P],
            "qc_cnn_flag": [_P, _P, _I64, _I64, _I32, _F, _I32, _P, _P],
        }.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        L.qc_channelize_set_variant.argtypes = [_I32]
        L.qc_channelize_set_variant.restype = ctypes.c_int32
        L.qc_channelize_get_variant.argtypes = []
        L.qc_channelize_get_variant.restype = ctypes.c_int32
        L.qc_xengine_set_variant.argtypes = [_I32]
        L.qc_xengine_set_variant.restype = ctypes.c_int32
        L.qc_xengine_get_variant.argtypes = []
        L.qc_xengine_get_variant.restype = ctypes.c_int32
        L.qc_measure_peak.argtypes = [_I32, ctypes.c_void_p, ctypes.c_int64, _I32,
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
        L.qc_measure_peak.restype = ctypes.c_int32
        L.qc_cnn_set_variant.argtypes = [_I32]
        L.qc_cnn_set_variant.restype = ctypes.c_int32
        L.qc_cnn_get_variant.argtypes = []
        L.qc_cnn_get_variant.restype = ctypes.c_int32
        L.qc_cnn_param_count.argtypes = []
        L.qc_cnn_param_count.restype = ctypes.c_int32
        L.qc_timing_enable.argtypes = [ctypes.c_int32]
        L.qc_timing_enable.restype = ctypes.c_int32
        L.qc_timing_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64)]
        L.qc_timing_read.restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != 0:
        L = lib()
        raise QCError(st, where, f"{L.qc_status_string(st).decode()}: {L.qc_last_error().decode()}")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Stream:
    """Streaming ingest: pinned host chunks -> device ring -> fused F+X with
    the filter history carried between chunks."""

    def __init__(self, n_ant, chunk_samp, n_fft, n_taps, spec_per_dump, depth=4):
        self.n_ant, self.chunk_samp, self.n_fft = n_ant, chunk_samp, n_fft
        self.spec_per_dump = spec_per_dump
        self._p = PfbParams(n_fft, n_taps, None, 0)
        h = ctypes.c_void_p()
        st = lib().qc_stream_create(n_ant, chunk_samp, ctypes.byref(self._p), spec_per_dump, depth,
                                    ctypes.byref(h))
        if st != 0:
            raise QCError(st, "qc_stream_create", lib().qc_stream_last_error().decode())
        self._h = h

    @property
    def n_dump_per_chunk(self):
        return (self.chunk_samp // self.n_fft) // self.spec_per_dump

    def push(self, host_chunk, seq, vis_out):
        """host_chunk: pinned int8 CPU tensor [n_ant, chunk_samp], or None for
        a dropped chunk (zero-filled); vis_out: device complex64."""
        if host_chunk is not None:
            assert host_chunk.dtype == torch.int8 and not host_chunk.is_cuda and host_chunk.is_contiguous()
        assert vis_out.is_cuda and vis_out.dtype == torch.complex64
        nd = _I64(0)
        ptr = None if host_chunk is None else ctypes.c_void_p(host_chunk.data_ptr())
        st = lib().qc_stream_push(self._h, ptr, seq, ctypes.c_void_p(vis_out.data_ptr()), ctypes.byref(nd))
        if st != 0:
            raise QCError(st, "qc_stream_push", lib().qc_stream_last_error().decode())
        return nd.value

    def valid_spectra(self):
        """Valid spectra per dump of the last pushed chunk (a list of ints)."""
        n = self.n_dump_per_chunk
        out = (_I64 * max(n, 1))()
        st = lib().qc_stream_valid_spectra(self._h, out, n)
        if st != 0:
            raise QCError(st, "qc_stream_valid_spectra", lib().qc_stream_last_error().decode())
        return list(out)[:n]

    def wait_copied(self, seq):
        st = lib().qc_stream_wait_copied(self._h, seq)
        if st != 0:
            raise QCError(st, "qc_stream_wait_copied", lib().qc_stream_last_error().decode())

    def sync(self):
        st = lib().qc_stream_sync(self._h)
        if st != 0:
            raise QCError(st, "qc_stream_sync", lib().qc_stream_last_error().decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().qc_stream_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Several arrays correlated together (qc_plan_*): per-array kernels on
    streams of their own, capturable as one hipGraph ("graph"), or every
    array's work in one persistent launch ("persistent")."""

    MODES = {"graph": 0, "persistent": 1}

    def __init__(self, arrays, mode="graph"):
        """arrays: list of dicts with n_ant, n_samp, n_fft, n_taps, spec_per_dump."""
        n = len(arrays)
        self.arrays = [dict(a) for a in arrays]
        descs = (ArrayDesc * n)(*[ArrayDesc(a["n_ant"], a["n_samp"], a["n_fft"], a.get("n_taps", 4),
                                            a["spec_per_dump"]) for a in arrays])
        h = ctypes.c_void_p()
        _check(lib().qc_plan_create(descs, n, ctypes.byref(h)), "qc_plan_create")
        self._h = h
        if mode != "graph":
            self.set_mode(mode)

    def set_mode(self, mode):
        _check(lib().qc_plan_set_mode(self._h, self.MODES[mode]), "qc_plan_set_mode")

    def empty_vis(self, device="cuda"):
        out = []
        for a in self.arrays:
            n_dump = (a["n_samp"] // a["n_fft"]) // a["spec_per_dump"]
            out.append(torch.empty((n_dump, n_base(a["n_ant"]), a["n_fft"] // 2),
                                   dtype=torch.complex64, device=device))
        return out

    @staticmethod
    def _ptrs(ts):
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def _call(self, name, xs, viss):
        for x in xs:
            _check_x(x)
            assert x.is_contiguous()
        _check(getattr(lib(), name)(self._h, self._ptrs(xs), self._ptrs(viss), _stream()), name)

    def execute(self, xs, viss):
        self._call("qc_plan_execute", xs, viss)

    def execute_separate(self, xs, viss):
        self._call("qc_plan_execute_separate", xs, viss)

    def capture_graph(self, xs, viss):
        self._call("qc_plan_capture_graph", xs, viss)

    def replay(self):
        _check(lib().qc_plan_replay(self._h, _stream()), "qc_plan_replay")

    def check(self):
        _check(lib().qc_plan_check(self._h, _stream()), "qc_plan_check")

    def set_wait_timeout(self, microseconds):
        _check(lib().qc_plan_set_wait_timeout(self._h, int(microseconds)), "qc_plan_set_wait_timeout")

    def set_wait_bias(self, n):
        _check(lib().qc_plan_set_wait_bias(self._h, n), "qc_plan_set_wait_bias")

    def autotune(self, xs, viss, reps=3, cache=None):
        fc = _I32(0)
        _check(lib().qc_plan_autotune(self._h, self._ptrs(xs), self._ptrs(viss), reps,
                                      None if cache is None else cache.encode(), ctypes.byref(fc),
                                      _stream()), "qc_plan_autotune")
        return bool(fc.value)

    def info(self):
        """(launches per execution, concurrent, per-array fused tile or -1, per-array split)."""
        n, c = _I32(0), _I32(0)
        m = len(self.arrays)
        tiles, splits = (_I32 * m)(), (_I64 * m)()
        _check(lib().qc_plan_info(self._h, ctypes.byref(n), ctypes.byref(c), tiles, splits),
               "qc_plan_info")
        return n.value, c.value, list(tiles), list(splits)

    def close(self):
        if getattr(self, "_h", None):
            lib().qc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def channelize_variant(v=None):
    """Get (and with v, set) the F-engine kernel choice: 0 ring where it applies, 1 plain."""
    if v is not None:
        _check(lib().qc_channelize_set_variant(int(v)), "qc_channelize_set_variant")
    return int(lib().qc_channelize_get_variant())


PEAK_KINDS = {"hbm_read": 0, "hbm_copy": 1, "valu_f32": 2, "mfma_f32": 3, "mfma_f16": 4}


def measure_peak(kind, scratch, reps=10):
    """Rate (GB/s or TFLOP/s) one measurement kernel of `kind` sustains on
    the current GPU; scratch: a CUDA tensor (its bytes are overwritten by
    the copy kind).  Not part of the method: a denominator for roofline
    fractions."""
    assert scratch.is_cuda and scratch.is_contiguous()
    rate = ctypes.c_double(0.0)
    st = lib().qc_measure_peak(PEAK_KINDS[kind], ctypes.c_void_p(scratch.data_ptr()),
                               scratch.numel() * scratch.element_size(), int(reps), ctypes.byref(rate),
                               _stream())
    _check(st, "qc_measure_peak")
    return rate.value


def cnn_variant(v=None):
    """Get (and with v, set) the flagger's float32 kernels (convolutions and
    weight gradients): 0 matrix cores, 1 vector ALU."""
    if v is not None:
        _check(lib().qc_cnn_set_variant(int(v)), "qc_cnn_set_variant")
    return int(lib().qc_cnn_get_variant())


def xengine_variant(v=None):
    """Get (and with v, set) the float32 X-engine kernel choice: 0 matrix cores
    for 5..32 antennas, 1 vector ALU, 2 matrix cores wherever supported."""
    if v is not None:
        _check(lib().qc_xengine_set_variant(int(v)), "qc_xengine_set_variant")
    return int(lib().qc_xengine_get_variant())


# ---- learned RFI flagger ----

def cnn_param_count():
    return int(lib().qc_cnn_param_count())


def _dev_f32(t, name):
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous(), name


def cnn_normalize(vis, out=None):
    """complex64 vis [n_time, n_base, n_chan] -> float32 images [n_base, n_time, n_chan]."""
    assert vis.dtype == torch.complex64 and vis.is_cuda and vis.is_contiguous()
    n_time, nb, n_chan = vis.shape
    if out is None:
        out = torch.empty((nb, n_time, n_chan), dtype=torch.float32, device=vis.device)
    _check(lib().qc_cnn_normalize(_ptr(vis), n_time, nb, n_chan, _ptr(out), _stream()), "qc_cnn_normalize")
    return out


ACT_PREC = {"f32": 0, "f16": 1}


def cnn_forward(params, x, out=None, act="f32"):
    """Logits [n, H, W] for normalised images x [n, H, W]; act "f16" runs
    half activations on the matrix cores."""
    _dev_f32(params, "params")
    _dev_f32(x, "x")
    n, H, W = x.shape
    if out is None:
        out = torch.empty_like(x)
    _check(lib().qc_cnn_forward(_ptr(params), _ptr(x), n, H, W, ACT_PREC[act], _ptr(out), _stream()),
           "qc_cnn_forward")
    return out


def cnn_grad(params, x, labels, pos_weight, grad=None, loss=None):
    """(grad [P], loss [1]) of the weighted BCE for images x and uint8 labels."""
    _dev_f32(params, "params")
    _dev_f32(x, "x")
    assert labels.is_cuda and labels.dtype == torch.uint8 and labels.shape == x.shape and labels.is_contiguous()
    n, H, W = x.shape
    if grad is None:
        grad = torch.empty_like(params)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(lib().qc_cnn_grad(_ptr(params), _ptr(x), _ptr(labels), n, H, W, float(pos_weight), _ptr(grad),
                             _ptr(loss), _stream()), "qc_cnn_grad")
    return grad, loss


def cnn_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().qc_cnn_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                             float(beta2), float(eps), _stream()), "qc_cnn_adam")


def cnn_train_step(params, m, v, step, x, labels, pos_weight, lr=1e-3, loss=None):
    n, H, W = x.shape
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(lib().qc_cnn_train_step(_ptr(params), _ptr(m), _ptr(v), int(step), _ptr(x), _ptr(labels), n, H, W,
                                   float(pos_weight), float(lr), _ptr(loss), _stream()), "qc_cnn_train_step")
    return loss


def cnn_flag(params, vis, threshold=0.0, mask=None, act="f32"):
    """uint8 mask [n_time, n_base, n_chan] from the network (logit > threshold)."""
    _dev_f32(params, "params")
    assert vis.dtype == torch.complex64 and vis.is_cuda and vis.is_contiguous()
    n_time, nb, n_chan = vis.shape
    if mask is None:
        mask = torch.empty(vis.shape, dtype=torch.uint8, device=vis.device)
    _check(lib().qc_cnn_flag(_ptr(params), _ptr(vis), n_time, nb, n_chan, float(threshold), ACT_PREC[act],
                             _ptr(mask), _stream()), "qc_cnn_flag")
    return mask


KERNELS = {"fx_fused": 0, "channelize": 1, "xeng_f32": 2, "xeng_mfma": 3, "reduce": 4,
           "mad": 5, "apply": 6}


def timing_enable(on=True):
    """Start (clearing) or stop per-kernel event timing inside the library.

    True: event pairs around each timed call; "chained": stop events bound to
    the launches themselves (no added packets; the stream must carry library
    calls only); False: off."""
    mode = 2 if on == "chained" else (1 if on else 0)
    _check(lib().qc_timing_enable(mode), "qc_timing_enable")


def timing_read(kernel: str):
    """(total milliseconds, launch count) recorded for a kernel; synchronises."""
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    _check(lib().qc_timing_read(KERNELS[kernel], ctypes.byref(ms), ctypes.byref(n)), "qc_timing_read")
    return ms.value, n.value


def solve_delay_phase(vis, n_ant, f0_hz, df_hz, ref_ant, chan_lo, chan_hi, mask=None, lag_pad=4):
    """Per-antenna (tau_s, phi_rad) numpy arrays from complex64 vis [n_time, n_base, n_chan]."""
    import numpy as np
    assert vis.dtype == torch.complex64 and vis.is_cuda and vis.is_contiguous()
    n_time, nb, n_chan = vis.shape
    assert nb == n_base(n_ant)
    if mask is not None:
        assert mask.dtype == torch.uint8 and mask.shape == vis.shape and mask.is_contiguous()
    tau = (ctypes.c_double * n_ant)()
    phi = (ctypes.c_double * n_ant)()
    _check(lib().qc_solve_delay_phase(_ptr(vis), _ptr(mask), n_time, n_ant, n_chan, float(f0_hz),
                                      float(df_hz), ref_ant, chan_lo, chan_hi, lag_pad, tau, phi,
                                      _stream()), "qc_solve_delay_phase")
    return np.array(list(tau)), np.array(list(phi))


def fx_tile_count(n_fft: int, n_ant: int) -> int:
    return lib().qc_fx_tile_count(n_fft, n_ant)


def fx_set_tile(n_fft: int, n_ant: int, tile: int):
    _check(lib().qc_fx_set_tile(n_fft, n_ant, tile), "qc_fx_set_tile")


def fx_get_tile(n_fft: int, n_ant: int) -> int:
    return lib().qc_fx_get_tile(n_fft, n_ant)


def fx_set_width(n_fft: int, n_ant: int, workgroups: int):
    """Workgroups per fused launch for (n_fft, n_ant); 0 restores the default."""
    _check(lib().qc_fx_set_width(n_fft, n_ant, workgroups), "qc_fx_set_width")


def fx_get_width(n_fft: int, n_ant: int) -> int:
    return lib().qc_fx_get_width(n_fft, n_ant)


def fx_autotune(x, n_fft, n_taps, spec_per_dump, reps=5):
    """Time every fused tile shape on x, then the fastest at other launch
    widths; keep the fastest; returns (best tile, [ms per tile])."""
    _check_x(x)
    n_ant, n_samp = x.shape
    n = fx_tile_count(n_fft, n_ant)
    n_dump = (n_samp // n_fft) // spec_per_dump
    vis = torch.empty((n_dump, n_base(n_ant), n_fft // 2), dtype=torch.complex64, device=x.device)
    ms = (ctypes.c_double * max(n, 1))()
    best = _I32(-1)
    p = PfbParams(n_fft, n_taps, None, 0)
    _check(lib().qc_fx_autotune(_ptr(x), x.stride(0), n_ant, n_samp, ctypes.byref(p), spec_per_dump,
                                reps, _ptr(vis), ms, n, ctypes.byref(best), _stream()), "qc_fx_autotune")
    return best.value, list(ms)[:n]


def n_base(n_ant: int) -> int:
    return n_ant * (n_ant + 1) // 2


def _pfb(n_fft, n_taps, taps):
    if taps is not None:
        assert taps.dtype == torch.float32 and taps.is_cuda and taps.numel() == n_fft * n_taps
    return PfbParams(n_fft, n_taps, None if taps is None else taps.data_ptr(), 0)


def _check_x(x):
    assert x.dtype == torch.int8 and x.is_cuda and x.dim() == 2 and x.stride(1) == 1, \
        "x must be a CUDA int8 [n_ant, n_samp] tensor with unit sample stride"


def _sample_word(x):
    """Input word of x: int8 / int16 [n_ant, n_samp] real, or int8 / int16
    [n_ant, n_samp, 2] complex (I, Q interleaved); returns (code, n_ant, n_samp, ld_x)."""
    assert x.is_cuda and x.dtype in (torch.int8, torch.int16), "x must be a CUDA int8 or int16 tensor"
    if x.dim() == 2:
        assert x.stride(1) == 1, "unit sample stride"
        return (0 if x.dtype == torch.int8 else 1), x.shape[0], x.shape[1], x.stride(0)
    assert x.dim() == 3 and x.shape[2] == 2 and x.stride(2) == 1 and x.stride(1) == 2, \
        "complex samples: [n_ant, n_samp, 2] with I, Q adjacent"
    assert x.stride(0) % 2 == 0
    return (2 if x.dtype == torch.int8 else 3), x.shape[0], x.shape[1], x.stride(0) // 2


def pfb_channelize_ex(x, n_fft, n_taps, taps=None, hist=None, hist_out=None, out_prec="f32",
                      out=None, scale_out=None):
    """F-engine of any input word (see _sample_word): (out, scale); out is
    complex64 [n_ant, n_spec, n_chan] for f32 (n_chan = N/2 real, N complex),
    else uint8 pairs of the format."""
    code, n_ant, n_samp, ld = _sample_word(x)
    prec = PREC[out_prec]
    n_spec = n_samp // n_fft
    n_chan = n_fft if code >= 2 else n_fft // 2
    if out is None:
        if prec == 0:
            out = torch.empty((n_ant, n_spec, n_chan), dtype=torch.complex64, device=x.device)
        else:
            out = torch.empty((n_ant, n_spec, n_chan * _PAIR_BYTES[prec]), dtype=torch.uint8, device=x.device)
    if prec != 0 and scale_out is None:
        scale_out = torch.empty(n_ant, dtype=torch.float32, device=x.device)
    p = _pfb(n_fft, n_taps, taps)
    _check(lib().qc_pfb_channelize_ex(_ptr(x), code, ld, n_ant, n_samp, ctypes.byref(p), _ptr(hist),
                                      _ptr(hist_out), prec, _ptr(out), _ptr(scale_out), _stream()),
           "qc_pfb_channelize_ex")
    return out, scale_out


def xcorrelate_ex(x, n_fft, n_taps, spec_per_dump, taps=None, hist=None, hist_out=None, vis=None,
                  accumulate=False, x_prec="f32"):
    """F+X of any input word: complex64 [n_dump, n_base, n_chan]."""
    code, n_ant, n_samp, ld = _sample_word(x)
    n_chan = n_fft if code >= 2 else n_fft // 2
    n_dump = (n_samp // n_fft) // spec_per_dump
    if vis is None:
        vis = torch.empty((n_dump, n_base(n_ant), n_chan), dtype=torch.complex64, device=x.device)
    p = _pfb(n_fft, n_taps, taps)
    nd = _I64(0)
    _check(lib().qc_xcorrelate_ex(_ptr(x), code, ld, n_ant, n_samp, ctypes.byref(p), _ptr(hist),
                                  _ptr(hist_out), spec_per_dump, PREC[x_prec], _ptr(vis),
                                  1 if accumulate else 0, ctypes.byref(nd), _stream()), "qc_xcorrelate_ex")
    assert nd.value == n_dump
    return vis


def design_taps(n_fft, n_taps, window="hann", beta=0.0, device="cuda"):
    """Prototype filter taps (float32 [P*N] on the device) from the library."""
    taps = torch.empty(n_fft * n_taps, dtype=torch.float32, device=device)
    _check(lib().qc_pfb_design_taps(n_fft, n_taps, WINDOW[window], float(beta), _ptr(taps), _stream()),
           "qc_pfb_design_taps")
    return taps


def ingest_run(paths, n_fft, n_taps, spec_per_dump, packet_samp, batch_packets, queue_max, n_readers=None,
               depth=4, sample="i8", taps=None, vis=None, max_dumps=-1):
    """File ingest (qc_ingest_run): one raw sample file per antenna, read by
    reader threads into queue_max pinned batch buffers, copied and
    correlated on the device.  Returns (vis complex64 [n_dump, n_base,
    n_chan], stats dict).  vis, if given, must hold max_dumps dumps."""
    n_ant = len(paths)
    code = SAMPLE[sample]
    wb = {0: 1, 1: 2, 2: 2, 3: 4}[code]
    n_chan = n_fft if code >= 2 else n_fft // 2
    batch_samp = packet_samp * batch_packets
    bspec = batch_samp // n_fft
    if vis is None:
        n_batch = min(os.path.getsize(p) for p in paths) // (batch_samp * wb)
        nd = (n_batch // (spec_per_dump // bspec)) if spec_per_dump >= bspec else n_batch * (bspec // spec_per_dump)
        if max_dumps >= 0:
            nd = min(nd, max_dumps)
        max_dumps = nd
        vis = torch.empty((max(nd, 1), n_base(n_ant), n_chan), dtype=torch.complex64, device="cuda")
    cfg = IngestConfig(n_ant, code, packet_samp, batch_packets, queue_max, n_readers or n_ant, depth,
                       _pfb(n_fft, n_taps, taps), spec_per_dump)
    arr = (ctypes.c_char_p * n_ant)(*[os.fsencode(p) for p in paths])
    st = IngestStats()
    _check(lib().qc_ingest_run(arr, ctypes.byref(cfg), _ptr(vis), max_dumps, ctypes.byref(st)), "qc_ingest_run")
    stats = {k: getattr(st, k) for k, _ in IngestStats._fields_}
    return vis[:st.dumps], stats


def image_grid(u, v, vis, n, cell_rad, weight=None, grid=None, wsum=None):
    """Nearest-cell gridding (qc_image_grid): returns (grid complex64 [n, n],
    wsum float64 [1]) on the device."""
    assert u.dtype == torch.float32 and v.dtype == torch.float32 and vis.dtype == torch.complex64
    n_vis = vis.numel()
    if grid is None:
        grid = torch.empty((n, n), dtype=torch.complex64, device=vis.device)
    if wsum is None:
        wsum = torch.empty(1, dtype=torch.float64, device=vis.device)
    _check(lib().qc_image_grid(_ptr(u), _ptr(v), _ptr(vis), _ptr(weight), n_vis, n, float(cell_rad),
                               _ptr(grid), _ptr(wsum), _stream()), "qc_image_grid")
    return grid, wsum


def image_invert(grid, wsum, image=None, work=None):
    """Dirty image (or beam) float32 [n, n] from a grid (qc_image_invert)."""
    n = grid.shape[0]
    if image is None:
        image = torch.empty((n, n), dtype=torch.float32, device=grid.device)
    if work is None:
        work = torch.empty((2, n, n), dtype=torch.complex64, device=grid.device)
    _check(lib().qc_image_invert(_ptr(grid), _ptr(wsum), n, _ptr(work), _ptr(image), _stream()),
           "qc_image_invert")
    return image


def image_dirty_and_psf(u, v, vis, n, cell_rad, weight=None):
    """(dirty image, synthesized beam), both float32 [n, n] on the device."""
    g, w = image_grid(u, v, vis, n, cell_rad, weight)
    dirty = image_invert(g, w)
    ones = torch.ones_like(vis)
    gp, wp = image_grid(u, v, ones, n, cell_rad, weight)
    return dirty, image_invert(gp, wp)


def image_clean(residual, psf, gain, threshold, max_iter):
    """Hogbom CLEAN in place on residual (qc_image_clean): returns
    (flat pixel indices int32 [k], fluxes float32 [k]) on the device."""
    n = residual.shape[0]
    assert residual.dtype == torch.float32 and psf.dtype == torch.float32 and residual.is_contiguous()
    pix = torch.empty(max(max_iter, 1), dtype=torch.int32, device=residual.device)
    flux = torch.empty(max(max_iter, 1), dtype=torch.float32, device=residual.device)
    nc = torch.empty(1, dtype=torch.int32, device=residual.device)
    _check(lib().qc_image_clean(_ptr(residual), _ptr(psf), n, float(gain), float(threshold), max_iter,
                                _ptr(pix), _ptr(flux), _ptr(nc), _stream()), "qc_image_clean")
    k = int(nc.item())
    return pix[:k], flux[:k]


def pfb_channelize(x, n_fft, n_taps, taps=None, hist=None, hist_out=None, out_prec="f32",
                   out=None, scale_out=None):
    """F-engine: returns (out, scale).  out is complex64 [n_ant, n_spec, n_chan]
    for f32, else a uint8 tensor holding (re, im) pairs of the format."""
    _check_x(x)
    n_ant, n_samp = x.shape
    prec = PREC[out_prec]
    n_spec, n_chan = n_samp // n_fft, n_fft // 2
    if out is None:
        if prec == 0:
            out = torch.empty((n_ant, n_spec, n_chan), dtype=torch.complex64, device=x.device)
        else:
            out = torch.empty((n_ant, n_spec, n_chan * _PAIR_BYTES[prec]), dtype=torch.uint8,
                              device=x.device)
    if prec != 0 and scale_out is None:
        scale_out = torch.empty(n_ant, dtype=torch.float32, device=x.device)
    p = _pfb(n_fft, n_taps, taps)
    st = lib().qc_pfb_channelize(_ptr(x), x.stride(0), n_ant, n_samp, ctypes.byref(p), _ptr(hist),
                                 _ptr(hist_out), prec, _ptr(out), _ptr(scale_out), _stream())
    _check(st, "qc_pfb_channelize")
    return out, scale_out


def xcorrelate(x, n_fft, n_taps, spec_per_dump, taps=None, hist=None, hist_out=None, vis=None,
               accumulate=False, x_prec="f32"):
    """Fused F+X: complex64 visibilities [n_dump, n_base, n_chan]."""
    _check_x(x)
    n_ant, n_samp = x.shape
    n_dump = (n_samp // n_fft) // spec_per_dump
    if vis is None:
        vis = torch.empty((n_dump, n_base(n_ant), n_fft // 2), dtype=torch.complex64, device=x.device)
    p = _pfb(n_fft, n_taps, taps)
    nd = _I64(0)
    st = lib().qc_xcorrelate(_ptr(x), x.stride(0), n_ant, n_samp, ctypes.byref(p), _ptr(hist),
                             _ptr(hist_out), spec_per_dump, PREC[x_prec], _ptr(vis),
                             1 if accumulate else 0, ctypes.byref(nd), _stream())
    _check(st, "qc_xcorrelate")
    assert nd.value == n_dump
    return vis


def xcorrelate_noalloc(x, n_fft, n_taps, spec_per_dump, vis, taps=None, hist=None, hist_out=None,
                       accumulate=False):
    """qc_xcorrelate_noalloc: the fused float32 F+X into a caller-supplied
    vis [n_dump, n_base, n_chan] (complex64); the library allocates nothing."""
    _check_x(x)
    n_ant, n_samp = x.shape
    n_dump = (n_samp // n_fft) // spec_per_dump
    assert vis.dtype == torch.complex64 and vis.is_contiguous()
    assert tuple(vis.shape) == (n_dump, n_base(n_ant), n_fft // 2)
    p = _pfb(n_fft, n_taps, taps)
    nd = _I64(0)
    st = lib().qc_xcorrelate_noalloc(_ptr(x), x.stride(0), n_ant, n_samp, ctypes.byref(p), _ptr(hist),
                                     _ptr(hist_out), spec_per_dump, _ptr(vis), 1 if accumulate else 0,
                                     ctypes.byref(nd), _stream())
    _check(st, "qc_xcorrelate_noalloc")
    assert nd.value == n_dump
    return vis


def xcorrelate_chan(v, prec, scale, n_ant, n_spec, n_chan, spec_per_dump, vis=None,
                    accumulate=False):
    """X-engine alone over channelised voltages laid out [n_ant][n_spec][n_chan]."""
    n_dump = n_spec // spec_per_dump
    if vis is None:
        vis = torch.empty((n_dump, n_base(n_ant), n_chan), dtype=torch.complex64, device=v.device)
    st = lib().qc_xcorrelate_chan(_ptr(v), PREC[prec], _ptr(scale), n_ant, n_spec, n_chan,
                                  spec_per_dump, _ptr(vis), 1 if accumulate else 0, _stream())
    _check(st, "qc_xcorrelate_chan")
    return vis


def mad_flag(vis, sigma=5.0, population=0, mask=None, thresh=None):
    """MAD flags for complex64 vis [n_time, n_base, n_chan]: (mask uint8, thresholds float64)."""
    assert vis.dtype == torch.complex64 and vis.is_cuda and vis.is_contiguous()
    n_time, nb, n_chan = vis.shape
    if mask is None:
        mask = torch.empty(vis.shape, dtype=torch.uint8, device=vis.device)
    tshape = {0: (nb,), 1: (nb, n_chan), 2: (n_time, nb)}[population]
    if thresh is None:
        thresh = torch.empty(tshape, dtype=torch.float64, device=vis.device)
    st = lib().qc_mad_flag(_ptr(vis), n_time, nb, n_chan, float(sigma), population, _ptr(mask),
                           _ptr(thresh), _stream())
    _check(st, "qc_mad_flag")
    return mask, thresh


def apply_delay_phase(vis, n_ant, f0_hz, df_hz, tau_s, phi_rad):
    """In-place delay/phase correction of complex64 vis [n_time, n_base, n_chan]."""
    assert vis.dtype == torch.complex64 and vis.is_cuda and vis.is_contiguous()
    n_time, nb, n_chan = vis.shape
    assert nb == n_base(n_ant)
    tau = (ctypes.c_double * n_ant)(*[float(v) for v in tau_s])
    phi = (ctypes.c_double * n_ant)(*[float(v) for v in phi_rad])
    st = lib().qc_apply_delay_phase(_ptr(vis), n_time, n_ant, n_chan, float(f0_hz), float(df_hz),
                                    tau, phi, _stream())
    _check(st, "qc_apply_delay_phase")
    return vis
