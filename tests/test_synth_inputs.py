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


def test_philox_known_answers():
    # Philox4x32-10 known-answer vectors published with the generator (Random123)
    from tacaw_synth.philox import philox4x32_10

    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF),
              (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        assert [int(x) for x in philox4x32_10(ctr, key)] == list(want)
    # vectorised counters give the scalar results
    r = philox4x32_10((np.arange(5), 7, 0, 0), (11, 0x21))
    for i in range(5):
        assert [int(x[i]) for x in r] == [int(x) for x in philox4x32_10((i, 7, 0, 0), (11, 0x21))]


def test_producer_twin_is_frame_range_independent():
    from tacaw_synth import philox as X

    spec = X.ProducerSpec(2, 200, 3, 5, seed=9)
    full = X.generate(spec)
    part = X.generate(spec, probes=[1], frames=(37, 151), pixels=[0, 4, 14])
    assert np.array_equal(part, full[[1]][:, 37:151][:, :, [0, 4, 14]])
    assert full.dtype == np.complex64
    # elastic 1 plus 8 tones of 1e-3/sqrt(8) plus noise
    assert 1e-4 < np.abs(full - 1).mean() < 3e-3
