"""Named plan shapes (paper_2607_02236_amd.workloads), host only.

Every preset's descriptor passes the library's host validation; the paper's
settings reproduce the numbers it prints (Sec. III.A: 31 chunks, 1.4 meV
sampling, 181 bins for +-30 THz, a 383-pixel +-100 mrad window; Sec. IV: 191
bins, 16 x 16 probes, detectors tiling 0-100 mrad); the benchmark presets'
masks are the synthetic series' four detectors."""

import numpy as np
import pytest

import tacaw_synth as T
from paper_2607_02236_amd import workloads as W


@pytest.mark.parametrize("name", list(W.PRESETS))
def test_every_preset_passes_host_validation(name):
    w = W.PRESETS[name]
    w.check()
    m = w.masks()
    assert m.shape == (len(w.detectors), w.ny, w.nx) and m.dtype == np.float64
    assert w.frames_used <= w.n_frames and w.n_segments >= 1
    if w.push_frames:
        assert w.n_frames % w.push_frames == 0
    if w.ring_frames:
        # deferred ring: room for every push beyond one chunk, a multiple of 64
        assert w.ring_frames % 64 == 0 and w.ring_frames - w.seg_len >= w.push_frames


def test_paper_plane_wave_numbers():
    w = W.PAPER_PLANE_WAVE
    assert w.n_segments == 31 and w.frames_used == w.n_frames  # "an average over 31 chunks"
    assert round(w.energy_step_mev, 1) == 1.4
    assert w.n_omega == 181  # the 181 x 383 x 383 result
    assert w.ny == w.nx == 383
    # 383 pixels at 0.52 mrad span the +-100 mrad window
    assert abs((w.nx - 1) / 2 * W.PAPER_MRAD_PER_PIXEL - 100) < 1.0


def test_paper_stem_numbers_and_detectors():
    w = W.PAPER_STEM
    assert w.n_probe == 256 and w.n_omega == 191 and w.max_probes_in_flight == 32
    m = w.masks()
    assert m.shape == (4, 383, 383)
    # the four detectors tile the disk theta < 100 mrad without overlap
    cy, cx = 383 // 2, 383 // 2
    y, x = np.meshgrid(np.arange(383) - cy, np.arange(383) - cx, indexing="ij")
    theta = np.sqrt(y * y + x * x) * W.PAPER_MRAD_PER_PIXEL
    total = m.sum(axis=0)
    assert total.max() == 1.0
    np.testing.assert_array_equal(total, (theta < 100.0 + 1e-9).astype(float))
    bf = m[0] > 0
    assert np.all(theta[bf] < 10.0 + 1e-9) and bf.sum() > 1000


@pytest.mark.parametrize("name,grid", [("realistic", 256), ("gradient", 128), ("streaming", 1024)])
def test_benchmark_masks_are_the_synthetic_four(name, grid):
    w = W.PRESETS[name]
    if grid > 256:
        # compare a band of rows through the centre (the full 1024^2 stack is 32 MB)
        m = w.masks()[:, 480:640]
        ref = T.standard_masks(grid, grid, scale=grid / 256)[:, 480:640]
    else:
        m, ref = w.masks(), T.standard_masks(grid, grid, scale=grid / 256)
    np.testing.assert_array_equal(m, ref)


def test_replace_keeps_the_rest():
    w = W.REALISTIC.replace(n_probe=4, transform="gemm_bf16x3", omega_half=62)
    assert (w.n_probe, w.transform, w.n_omega, w.seg_len) == (4, "gemm_bf16x3", 125, 512)
    w.check()
    assert W.REALISTIC.n_probe == 64
