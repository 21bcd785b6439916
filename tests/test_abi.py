"""The C-ABI library: loads, exports every declared symbol, rejects bad
arguments on the host before any launch.  CPU only (no compute calls)."""

import ctypes
import os

import pytest

from tests.util import header_functions

import paper_2604_20640_amd as qc

pytestmark = pytest.mark.skipif(not os.path.exists(qc.LIB_PATH), reason="libqc.so not built")

QC_EINVAL, QC_EUNSUPPORTED = -1, -2


def test_exports_every_header_symbol():
    names = header_functions()
    assert len(names) >= 8
    L = ctypes.CDLL(qc.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_version():
    L = qc.lib()
    assert L.qc_status_string(0) == b"QC_OK"
    assert L.qc_status_string(-1) == b"QC_EINVAL"
    assert b"gfx950" in L.qc_version()


def _params(n_fft=1024, n_taps=4, taps=None, keep=0):
    return qc.PfbParams(n_fft, n_taps, taps, keep)


def _xcorr(x=0x1000, ld=4096, n_ant=4, n_samp=4096, p=None, hist=None, hist_out=None, spd=1,
           prec=0, vis=0x2000, acc=0):
    p = p or _params()
    nd = ctypes.c_int64(-7)
    st = qc.lib().qc_xcorrelate(ctypes.c_void_p(x), ld, n_ant, n_samp, ctypes.byref(p),
                                ctypes.c_void_p(hist) if hist else None,
                                ctypes.c_void_p(hist_out) if hist_out else None, spd, prec,
                                ctypes.c_void_p(vis) if vis else None, acc, ctypes.byref(nd), None)
    return st


@pytest.mark.parametrize("kw", [
    dict(p=_params(n_fft=1000)),            # not a power of two
    dict(p=_params(n_fft=2)),               # too small
    dict(p=_params(n_fft=16384)),           # too large
    dict(p=_params(n_taps=0)),
    dict(p=_params(n_taps=17)),
    dict(n_samp=4095),                      # not a multiple of N
    dict(ld=4095),                          # ld_x not multiple of 4
    dict(ld=1024),                          # ld_x < n_samp
    dict(n_ant=0),
    dict(spd=0),
    dict(x=0x1001),                         # misaligned x
    dict(hist=0x3000, hist_out=0x3000),     # aliasing history
    dict(prec=7),
    dict(vis=0x2004),                       # misaligned vis
    dict(vis=0),                            # vis NULL with a full dump
    dict(x=0),                              # x NULL
    dict(p=_params(taps=0x1004)),           # misaligned user taps
])
def test_xcorrelate_rejects(kw):
    assert _xcorr(**kw) == QC_EINVAL
    assert qc.lib().qc_last_error() != b""


def test_keep_nyquist_unsupported():
    assert _xcorr(p=_params(keep=1)) == QC_EUNSUPPORTED


def test_channelize_rejects():
    L = qc.lib()
    p = _params()
    st = L.qc_pfb_channelize(ctypes.c_void_p(0x1000), 4096, 4, 4096, ctypes.byref(p), None, None,
                             1, ctypes.c_void_p(0x2000), None, None)   # no scale_out for f16
    assert st == QC_EINVAL
    st = L.qc_pfb_channelize(ctypes.c_void_p(0x1000), 4096, 4, 4096, ctypes.byref(p), None, None,
                             0, None, None, None)                       # out NULL
    assert st == QC_EINVAL
    st = L.qc_pfb_channelize(ctypes.c_void_p(0x1000), 4096, 4, 4096, None, None, None, 0,
                             ctypes.c_void_p(0x2000), None, None)       # params NULL
    assert st == QC_EINVAL


def test_mad_rejects():
    L = qc.lib()
    v, m = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert L.qc_mad_flag(v, 4, 3, 8, 5.0, 3, m, None, None) == QC_EINVAL          # population
    assert L.qc_mad_flag(v, 0, 3, 8, 5.0, 0, m, None, None) == QC_EINVAL          # n_time 0
    assert L.qc_mad_flag(v, 4, 3, 8, float("nan"), 0, m, None, None) == QC_EINVAL  # sigma
    assert L.qc_mad_flag(v, 4, 3, 8, -1.0, 0, m, None, None) == QC_EINVAL
    assert L.qc_mad_flag(None, 4, 3, 8, 5.0, 0, m, None, None) == QC_EINVAL
    assert L.qc_mad_flag(ctypes.c_void_p(0x1004), 4, 3, 8, 5.0, 0, m, None, None) == QC_EINVAL


def test_apply_rejects():
    L = qc.lib()
    d2 = ctypes.c_double * 2
    t, p = d2(0.0, 1e-9), d2(0.0, 0.5)
    v = ctypes.c_void_p(0x1000)
    assert L.qc_apply_delay_phase(v, 1, 65, 8, 0.0, 1.0, t, p, None) == QC_EINVAL
    assert L.qc_apply_delay_phase(v, 1, 2, 0, 0.0, 1.0, t, p, None) == QC_EINVAL
    assert L.qc_apply_delay_phase(v, 1, 2, 8, float("inf"), 1.0, t, p, None) == QC_EINVAL
    bad = d2(0.0, float("nan"))
    assert L.qc_apply_delay_phase(v, 1, 2, 8, 0.0, 1.0, bad, p, None) == QC_EINVAL
    assert L.qc_apply_delay_phase(None, 1, 2, 8, 0.0, 1.0, t, p, None) == QC_EINVAL
    assert L.qc_apply_delay_phase(v, 1, 2, 8, 0.0, 1.0, None, p, None) == QC_EINVAL
    # zero time samples is a valid no-op that touches nothing
    assert L.qc_apply_delay_phase(None, 0, 2, 8, 0.0, 1.0, t, p, None) == 0


def test_zero_dumps_is_noop():
    # fewer spectra than one dump and no history output: nothing to launch
    nd = ctypes.c_int64(-1)
    p = _params()
    st = qc.lib().qc_xcorrelate(ctypes.c_void_p(0x1000), 4096, 4, 4096, ctypes.byref(p), None, None,
                                8, 0, None, 0, ctypes.byref(nd), None)
    assert st == 0 and nd.value == 0


def test_kernel_variant_switches():
    # host-side state only: range checks and round trips, defaults restored
    L = qc.lib()
    assert L.qc_xengine_get_variant() == 0 and L.qc_channelize_get_variant() == 0
    for bad in (-1, 3):
        assert L.qc_xengine_set_variant(bad) == QC_EINVAL
    assert L.qc_channelize_set_variant(2) == QC_EINVAL
    try:
        for v in (1, 2, 0):
            assert L.qc_xengine_set_variant(v) == 0 and L.qc_xengine_get_variant() == v
    finally:
        L.qc_xengine_set_variant(0)
    assert qc.xengine_variant() == 0
    assert L.qc_cnn_get_variant() == 0
    for bad in (-1, 2):
        assert L.qc_cnn_set_variant(bad) == QC_EINVAL
    try:
        assert L.qc_cnn_set_variant(1) == 0 and qc.cnn_variant() == 1
    finally:
        L.qc_cnn_set_variant(0)
    assert qc.cnn_variant() == 0


def test_fused_width_setting():
    # host-side state only: range checks and round trips, default restored
    L = qc.lib()
    assert L.qc_fx_get_width(4096, 4) == 0
    assert L.qc_fx_set_width(4096, 4, -1) == QC_EINVAL
    assert L.qc_fx_set_width(4096, 4, (1 << 20) + 1) == QC_EINVAL
    assert L.qc_fx_set_width(4096, 3, 256) == QC_EUNSUPPORTED    # no fused kernel
    try:
        assert L.qc_fx_set_width(4096, 4, 256) == 0 and qc.fx_get_width(4096, 4) == 256
        assert qc.fx_get_width(1024, 4) == 0                       # per (n_fft, n_ant)
    finally:
        assert L.qc_fx_set_width(4096, 4, 0) == 0
    assert qc.fx_get_width(4096, 4) == 0


def test_measure_peak_rejects_bad_arguments():
    # host-side validation only: no GPU work is started
    L = qc.lib()
    r = ctypes.c_double(0.0)
    p = ctypes.c_void_p(0x100000)
    assert L.qc_measure_peak(5, p, 1 << 30, 1, ctypes.byref(r), None) == QC_EINVAL    # unknown kind
    assert L.qc_measure_peak(-1, p, 1 << 30, 1, ctypes.byref(r), None) == QC_EINVAL
    assert L.qc_measure_peak(0, None, 1 << 30, 1, ctypes.byref(r), None) == QC_EINVAL  # null scratch
    assert L.qc_measure_peak(0, p, 1 << 30, 1, None, None) == QC_EINVAL                # null rate
    assert L.qc_measure_peak(0, p, 1 << 30, 0, ctypes.byref(r), None) == QC_EINVAL     # reps < 1
    assert L.qc_measure_peak(0, ctypes.c_void_p(0x100008), 1 << 30, 1, ctypes.byref(r), None) == QC_EINVAL
    assert L.qc_measure_peak(1, p, (64 << 20) - 32, 1, ctypes.byref(r), None) == QC_EINVAL  # too small
    assert L.qc_measure_peak(3, p, (64 << 10) - 16, 1, ctypes.byref(r), None) == QC_EINVAL

