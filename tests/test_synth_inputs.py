"""Host checks of the seeded input generator (shared by oracle and GPU path)."""

import numpy as np
import torch

import tacaw_synth as T


def test_subset_and_frame_ranges_are_bit_identical():
    spec = T.config_realistic(n_probe=3, n_frames=96, ny=16, nx=24, seed=9)
    full = T.generate(spec).reshape(3, 96, -1)
    pix = np.array([0, 7, 100, 383])
    assert torch.equal(T.generate(spec, probes=[2, 0], pixels=pix), full[[2, 0]][:, :, pix])
    assert torch.equal(T.generate(spec, frames=(31, 77)).reshape(3, 46, -1), full[:, 31:77])


def test_seeded_and_structured():
    a = T.generate(T.config_plain_1probe())
    b = T.generate(T.config_plain_1probe())
    assert torch.equal(a, b) and a.dtype == torch.complex128
    spec = T.SeriesSpec(1, 64, 4, 4, seed=3, noise_sigma=0.0, n_terms=0)
    assert torch.all(T.generate(spec) == 1.0)
    c = T.generate(T.SeriesSpec(1, 64, 4, 4, seed=4)) - 1.0
    assert 1e-4 < c.abs().mean() < 5e-3


def test_masks_and_weights():
    m = T.standard_masks(256, 256)
    assert m.shape == (4, 256, 256)
    assert m[0, 128, 128] == 1 and m[1, 128, 128] == 0 and m[1, 128, 128 + 80] == 1
    assert m[2, 128, 188] == 1 and m[3, 188, 128] == 1
    ann = T.disk_mask(64, 64, 24, inner=8)
    assert ann[32, 32 + 8] == 1 and ann[32, 32 + 7] == 0 and ann[32, 32 + 23] == 1 and ann[32, 32 + 24] == 0
    a = T.loss_weights(4, 16)
    assert a.shape == (4, 16) and np.all(a[3] <= 0.125)


def test_non_stationary_series():
    spec = T.SeriesSpec(2, 40, 2, 8, seed=5, noise_sigma=0.0, n_terms=0)  # psi == 1
    psi = T.generate(spec)
    off = T.perturb(psi, "offset", 0.2)
    assert off.dtype == psi.dtype
    assert torch.allclose(off[:, 0], torch.full_like(off[:, 0], 1.2))
    assert torch.equal(off[:, 1:], psi[:, 1:])
    tr = T.perturb(psi, "transient", 0.5, tau=4.0)
    assert abs(float(tr[0, 8, 0, 0].real) - (1.0 + 0.5 * np.exp(-2.0))) < 1e-7
    dr = T.perturb(psi, "drift", 0.01)
    # phase advance per frame = 2 pi f(kx), f = 0.01 (kx - 4) / 4; |psi| unchanged
    assert torch.allclose(dr.abs(), psi.abs())
    ph = np.angle(dr[0, 1, 0].numpy())
    assert np.allclose(ph, 2 * np.pi * 0.01 * (np.arange(8) - 4) / 4, atol=1e-6)
