"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/tacaw.h declares, and validates descriptors without touching a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tacaw.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tacaw_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("tacaw_plan", "tacaw_push_frames", "tacaw_finalize", "tacaw_detector_spectra",
              "tacaw_backward", "tacaw_destroy", "tacaw_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2607_02236_amd import tacaw

    lib = ctypes.CDLL(tacaw.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(tacaw.EXPORTED) == set(declared_functions())


def _ok(**over):
    kw = dict(n_probe=2, ny=8, nx=8, n_frames=256, seg_len=128, hop=64)
    kw.update(over)
    return kw


@pytest.mark.parametrize("over,kind", [
    (dict(hop=0), "INVALID_ARG"),
    (dict(hop=129), "INVALID_ARG"),
    (dict(n_frames=100), "INVALID_ARG"),
    (dict(seg_len=100), "UNSUPPORTED"),
    (dict(seg_len=200, hop=100, n_frames=400, transform="gemm_bf16x3"), "UNSUPPORTED"),
    (dict(seg_len=2048, n_frames=4096), "UNSUPPORTED"),
    (dict(n_probe=0), "INVALID_ARG"),
    (dict(ny=0), "INVALID_ARG"),
    (dict(window="hann_width", window_param=0.0), "INVALID_ARG"),
    (dict(window="tukey", window_param=1.5), "INVALID_ARG"),
    (dict(mean_mode="per_segment", transform="gemm_f16x3"), "UNSUPPORTED"),
    (dict(mean_mode="per_segment", hop=31), "UNSUPPORTED"),  # more than 4 chunks per frame
    (dict(dt_fs=0.0), "INVALID_ARG"),
    (dict(n_det=2), "INVALID_ARG"),
    (dict(max_probes_in_flight=3), "INVALID_ARG"),
    (dict(ny=1 << 16, nx=1 << 16), "INVALID_ARG"),
    (dict(window="custom"), "INVALID_ARG"),
    (dict(temperature_K=-1.0), "INVALID_ARG"),
    (dict(omega_half=-1), "INVALID_ARG"),
    (dict(k_row_stride=7), "INVALID_ARG"),    # k window: row stride below nx
    (dict(ring_frames=128), "INVALID_ARG"),   # must exceed seg_len
    (dict(ring_frames=160), "INVALID_ARG"),   # multiple of seg_len / 2
    (dict(ring_frames=256, transform="gemm_f16x3"), "UNSUPPORTED"),
    (dict(omega_half=64), "INVALID_ARG"),  # must be < seg_len / 2
    (dict(flags=2), "INVALID_ARG"),                           # tiled ring without a ring
    (dict(flags=2, ring_frames=256, hop=128, n_frames=512), "UNSUPPORTED"),  # needs hop = L/2
])
def test_descriptor_validation_errors(over, kind):
    from paper_2607_02236_amd import tacaw

    with pytest.raises(tacaw.TacawError) as e:
        tacaw.check_desc(**_ok(**over))
    assert e.value.kind == kind
    assert tacaw.lib.tacaw_last_error().decode()


def test_valid_descriptors_pass():
    from paper_2607_02236_amd import tacaw

    tacaw.check_desc(**_ok())
    tacaw.check_desc(**_ok(window="rect", mean_mode="none", in_dtype="c128", probe_reduce="sum"))
    tacaw.check_desc(**_ok(seg_len=1024, n_frames=4096, hop=512, max_probes_in_flight=1))
    import numpy as np

    tacaw.check_desc(**_ok(window=np.hanning(128), temperature_K=300.0))
    tacaw.check_desc(**_ok(transform="gemm_bf16x3"))
    tacaw.check_desc(**_ok(omega_half=63))
    tacaw.check_desc(**_ok(ring_frames=192))
    tacaw.check_desc(**_ok(ring_frames=192, flags=tacaw.FLAG_TILED_RING))
    tacaw.check_desc(**_ok(k_row_stride=40))
    tacaw.check_desc(**_ok(mean_mode="per_segment", hop=32))
    tacaw.check_desc(**_ok(mean_mode="per_segment", ring_frames=192, flags=tacaw.FLAG_TILED_RING))
    tacaw.check_desc(**_ok(seg_len=200, hop=100, n_frames=3200, dt_fs=15.0, omega_half=90))
    tacaw.check_desc(**_ok(omega_half=1, transform="gemm_f16x3", temperature_K=50.0))
    tacaw.check_desc(**_ok(transform="gemm_f16x3", seg_len=1024, n_frames=2048, hop=512))
    tacaw.check_desc(**_ok(transform="gemm_bf16x3", ring_frames=192, flags=tacaw.FLAG_TILED_RING))


def test_null_arguments_are_rejected_without_a_device():
    from paper_2607_02236_amd import tacaw

    lib = tacaw.lib
    assert lib.tacaw_plan_check(None) == -1
    h = ctypes.c_void_p()
    assert lib.tacaw_plan(None, None, ctypes.byref(h)) == -1 and not h.value
    assert lib.tacaw_push_frames(None, None, 0, 1, 1, 1, 1) == -1
    assert lib.tacaw_finalize(None, None) == -1
    assert lib.tacaw_detector_spectra(None, None, 0, None, None) == -1
    assert lib.tacaw_reset(None) == -1
    n = ctypes.c_int64(0)
    assert lib.tacaw_plan_export(None, None, 0, ctypes.byref(n)) == -1
    assert lib.tacaw_plan_import(None, b"\0" * 64, 64) == -1
    assert lib.tacaw_read_probe(None, 16, None, None) == -1
    lib.tacaw_destroy(None)


def test_axes_helpers_match_paper_numbers():
    import numpy as np

    from paper_2607_02236_amd import axes

    assert len(axes.roi_bins(200, 15.0, 30.0)) == 181
    # the 181-bin window of +-30 THz at L = 200, 15 fs as a plan's omega_half
    M = axes.omega_half_for(200, 15.0, f_max_thz=30.0)
    assert 2 * M + 1 == 181
    np.testing.assert_array_equal(np.sort(axes.window_rows(200, M)), axes.roi_bins(200, 15.0, 30.0))
    assert axes.omega_half_for(512, 5.0, e_max_mev=100.0) == 61  # 100 meV / 1.6155 meV
    assert axes.omega_half_for(256, 5.0, f_max_thz=1e9) == 127
    np.testing.assert_array_equal(axes.window_rows(8, 0), np.arange(8))
    np.testing.assert_array_equal(axes.window_rows(8, 2), [6, 7, 0, 1, 2])
    assert round(axes.energy_step_mev(200, 15.0), 1) == 1.4
    e = axes.energy_mev(256, 5.0)
    assert e[1] > 0 and e[255] < 0 and abs(e[128]) == pytest.approx(413.567, rel=1e-5)


def test_detector_helpers_match_input_masks():
    import numpy as np

    import tacaw_synth as T
    from paper_2607_02236_amd import detectors

    np.testing.assert_array_equal(detectors.annular(64, 64, 8, 24), T.disk_mask(64, 64, 24, inner=8))
    ds = detectors.detector_set(256, 256,
                                {"type": "circular", "radius": 30},
                                {"type": "annular", "radius_inner": 60, "radius_outer": 100},
                                {"type": "circular", "center": (128, 188), "radius": 30},
                                {"type": "circular", "center": (188, 128), "radius": 30})
    np.testing.assert_array_equal(ds, T.standard_masks(256, 256))
