"""CPU-side checks of the C ABI: the library builds, loads and exports every
symbol declared in include/rsfstat.h; the ctypes mirror has the header's
layout.  No compute call is made (there is no GPU here)."""
import ctypes as C
import os
import re

import pytest

from paper_0912_4255_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsfstat.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(rsf_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_0912_4255_amd import build
        build.build()
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    assert set(names) == set(L.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_error_string(lib):
    assert lib.rsf_version() == 1
    assert isinstance(lib.rsf_last_error(), bytes)


def test_struct_sizes_match_header_layout():
    # rsf_plan_desc: 6 int32 + int64 + 5 double + ephemeris (7 double) + 4 detectors (4 double)
    assert C.sizeof(L.PlanDesc) == 6 * 4 + 8 + 5 * 8 + 7 * 8 + 4 * 4 * 8
    assert C.sizeof(L.Segment) == 4 * 8 + 4 * 8 + 4 * 4
    assert C.sizeof(L.Resampled) == 7 * 8
    assert C.sizeof(L.TopkEntry) == 16
    # rsf_sft_desc: 5 int64 + 6 double + 2 int32
    assert C.sizeof(L.SftDesc) == 5 * 8 + 6 * 8 + 2 * 4
    # rsf_hetdec_desc: int64, 2 double, 2 int32, double, int64
    assert C.sizeof(L.HetdecDesc) == 8 + 2 * 8 + 2 * 4 + 8 + 8


def test_null_arguments_rejected_without_gpu(lib):
    p = C.c_void_p()
    assert lib.rsf_plan_create(C.byref(p), None) == L.RSF_EINVAL
    assert b"NULL" in lib.rsf_last_error()
    b = C.c_size_t()
    assert lib.rsf_workspace_size(None, 0, 1, 1, 0, C.byref(b)) == L.RSF_EINVAL
    assert lib.rsf_fstat(None, None, None, 1, None, 1, 0, None, None, 0, None) == L.RSF_EINVAL
    assert lib.rsf_plan_batching(None, 1, 1, 0, None, None, None) == L.RSF_EINVAL


def test_multi_segment_arguments_rejected_without_gpu(lib):
    b = C.c_size_t()
    assert lib.rsf_segments_workspace_size(None, 1, 1, 1, C.byref(b)) == L.RSF_EINVAL
    plans = (C.c_void_p * 2)(None, None)
    assert lib.rsf_segments_workspace_size(plans, 2, 1, 1, C.byref(b)) == L.RSF_EINVAL
    assert b"plans[0]" in lib.rsf_last_error()
    assert lib.rsf_segments_workspace_size(plans, 0, 1, 1, C.byref(b)) == L.RSF_EINVAL
    assert lib.rsf_fstat_topk_segments(None, None, 1, None, 1, None, 1, 10, None, None, 0, None) == L.RSF_EINVAL
    g = C.c_void_p()
    assert lib.rsf_graph_create_topk_segments(C.byref(g), plans, None, 2, None, 1, None, 1, 10, None, None, 0) == \
        L.RSF_EINVAL
    assert not g.value


def test_invalid_descriptors_rejected_before_device_use(lib):
    from paper_0912_4255_amd import synth
    from paper_0912_4255_amd.api import plan_desc_from_workload
    w = synth.small_workload(n=1000, dt=1.0)
    cases = []
    d = plan_desc_from_workload(w); d.taps = 7; cases.append((d, L.RSF_EUNSUPPORTED))
    d = plan_desc_from_workload(w); d.taps = 40; cases.append((d, L.RSF_EUNSUPPORTED))
    d = plan_desc_from_workload(w); d.dt = -1.0; cases.append((d, L.RSF_EINVAL))
    d = plan_desc_from_workload(w); d.n = 0; cases.append((d, L.RSF_EINVAL))
    d = plan_desc_from_workload(w); d.n_det = 0; cases.append((d, L.RSF_EINVAL))
    d = plan_desc_from_workload(w); d.det[0].sigma2 = 0.0; cases.append((d, L.RSF_EINVAL))
    d = plan_desc_from_workload(w); d.f_het = float("nan"); cases.append((d, L.RSF_EINVAL))
    d = plan_desc_from_workload(w); d.n = 1001; cases.append((d, L.RSF_EUNSUPPORTED))   # 2002 = 2 * 7 * 11 * 13
    d = plan_desc_from_workload(w); d.f_lo, d.f_hi = 99.0, 99.2; cases.append((d, L.RSF_EINVAL))
    d = plan_desc_from_workload(w); d.fft_l1 = -5; cases.append((d, L.RSF_EINVAL))
    for desc, code in cases:
        p = C.c_void_p()
        assert lib.rsf_plan_create(C.byref(p), C.byref(desc)) == code, lib.rsf_last_error()
        assert not p.value


def test_fft_factorisation_covers_every_workload_length(lib):
    """Every FFT length of the standard workloads, and of all 64 uneven
    segments (even 7-smooth lengths, and 7-smooth multiples of 256), has a
    two-pass factorisation that fits 160 KiB of LDS, with a one-column-per-
    wave second pass wherever one fits; non-7-smooth lengths are refused."""
    from oracle.fstat import NFFT_SMOOTH7, NFFT_SMOOTH7_256, fft_length
    from paper_0912_4255_amd.synth import c3_segment_lengths
    lengths = [345600, 6912000, 10368000, 3456000]
    lengths += [fft_length(n, NFFT_SMOOTH7) for n in c3_segment_lengths()]
    lengths += [fft_length(n, NFFT_SMOOTH7_256) for n in c3_segment_lengths()]
    for m in lengths:
        l1, l2 = C.c_int32(), C.c_int32()
        assert lib.rsf_fft_factor(m, 163840, 0, C.byref(l1), C.byref(l2)) == L.RSF_OK, (m, lib.rsf_last_error())
        assert l1.value * l2.value == m and l1.value <= 10240
    # the one-column-per-wave second pass (L2 = 256, 512, 768) is preferred
    # where it fits, then L2 = 1024 (one column per wave for the top-k)
    l1, l2 = C.c_int32(), C.c_int32()
    assert lib.rsf_fft_factor(6912000, 163840, 0, C.byref(l1), C.byref(l2)) == L.RSF_OK
    assert (l1.value, l2.value) == (9000, 768)

    def first_pass_fits(la):   # the row and its two-level twiddle table in 160 KiB
        return la <= 10240 and la * 16 + (32 + (la + 31) // 32) * 8 <= 163840

    wave = wave16 = 0
    for n in c3_segment_lengths():
        m = fft_length(n, NFFT_SMOOTH7_256)
        assert lib.rsf_fft_factor(m, 163840, 0, C.byref(l1), C.byref(l2)) == L.RSF_OK
        wave += l2.value in (256, 512, 768)
        wave16 += l2.value == 1024
        if any(m % lb == 0 and m // lb <= 10000 for lb in (256, 512, 768)):
            assert l2.value in (256, 512, 768), (m, l1.value, l2.value)
        elif m % 1024 == 0 and first_pass_fits(m // 1024):
            assert l2.value == 1024, (m, l1.value, l2.value)
    assert wave >= 45 and wave + wave16 >= 56
    assert lib.rsf_fft_factor(2 * 11 * 1000, 163840, 0, None, None) == L.RSF_EUNSUPPORTED
    assert lib.rsf_fft_factor(6912000, 163840, 7200, C.byref(l1), None) == L.RSF_OK and l1.value == 7200



def test_invalid_sft_descriptors_rejected_before_device_use(lib):
    """The SFT front end checks its descriptor and start times on the host
    before any device call: B T_sft even, f_h T_sft whole, f_h >= B/2, odd
    median window within the band, increasing start times on the output grid."""
    import numpy as np
    from paper_0912_4255_amd import synth
    from paper_0912_4255_amd.api import sft_desc_from_set
    ss = synth.SftSet(sft_len=256, dt_raw=1.0 / 64.0, k_lo=30, n_bins=200, t_sft=np.arange(4) * 4.0, t_start=0.0,
                      f_het=10.25, band=2.0, n_out=64, dk=8, median_window=51)
    t_ok = np.ascontiguousarray(ss.t_sft)
    cases = []
    d = sft_desc_from_set(ss); d.band = 2.25; cases.append((d, t_ok))             # B T_sft = 9, odd
    d = sft_desc_from_set(ss); d.f_het = 10.1; cases.append((d, t_ok))            # f_h T_sft = 40.4
    d = sft_desc_from_set(ss); d.f_het = 0.75; cases.append((d, t_ok))            # below B/2
    d = sft_desc_from_set(ss); d.median_window = 50; cases.append((d, t_ok))
    d = sft_desc_from_set(ss); d.median_window = 201; cases.append((d, t_ok))     # wider than the band
    d = sft_desc_from_set(ss); d.dk = 17; cases.append((d, t_ok))
    d = sft_desc_from_set(ss); d.band_taper = 1.5; cases.append((d, t_ok))
    d = sft_desc_from_set(ss); cases.append((d, np.array([0.0, 4.0, 4.0, 8.0])))  # not increasing
    d = sft_desc_from_set(ss); cases.append((d, np.array([0.0, 4.0, 8.3, 12.3])))  # off the output grid
    for desc, t in cases:
        p = C.c_void_p()
        t = np.ascontiguousarray(t, dtype=np.float64)
        rc = lib.rsf_sft_plan_create(C.byref(p), C.byref(desc), t.ctypes.data_as(C.POINTER(C.c_double)))
        assert rc == L.RSF_EINVAL, lib.rsf_last_error()
        assert not p.value


def test_invalid_hetdec_descriptors_rejected_before_device_use(lib):
    good = dict(n_raw=1000, dt_raw=1.0 / 256.0, f_het=100.0, D=64, K=16, beta=8.0, n_out=10)
    bad = [dict(D=0), dict(K=-1), dict(beta=-1.0), dict(dt_raw=0.0), dict(n_out=0), dict(f_het=float("inf")),
           dict(D=512, K=16)]                       # taps and tile beyond 160 KiB of LDS
    for b in bad:
        d = dict(good)
        d.update(b)
        desc = L.HetdecDesc(d["n_raw"], d["dt_raw"], d["f_het"], d["D"], d["K"], d["beta"], d["n_out"])
        p = C.c_void_p()
        rc = lib.rsf_hetdec_plan_create(C.byref(p), C.byref(desc))
        assert rc in (L.RSF_EINVAL, L.RSF_EUNSUPPORTED), (b, lib.rsf_last_error())
        assert not p.value
