"""The paper's own run settings at their full k-grid, against the FP64 oracle.

Sec. III.A's plane-wave window study: one probe, 31 Welch chunks of 200
snapshots at 15 fs (hop 100, 3200 frames), a 383 x 383 k-space window and the
+-30 THz energy window (181 bins). Sec. IV's STEM scan: the same grid and
chunking, 191 bins, probes pushed in batches and the four detectors of 0-10,
10-30, 30-60 and 60-100 mrad (here 8 of its 256 probes, in batches of 4).

The exit waves come from the fused producer (Philox4x32-10) in pieces of 200
frames, pushed as they are made; its CPU twin regenerates sampled pixels bit for
bit, on which the oracle computes S, and the detector masks are restricted to
those pixels so that D and D_p are checked against the oracle too. The grid has
146,689 pixels: 4,584 full 32-pixel tiles of the L = 200 kernel and a last tile
of one pixel, which is always sampled."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_02236_amd import axes, detectors
from paper_2607_02236_amd import workloads as W
from tacaw_synth import philox as X

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = float(np.linalg.norm(np.ravel(b)))
    d = float(np.linalg.norm(np.ravel(a) - np.ravel(b)))
    return d / nb if nb > 0 else d


@pytest.fixture(scope="module")
def tacaw():
    from paper_2607_02236_amd import tacaw as t

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return t


def producer(tacaw, w, seed):
    spec = X.ProducerSpec(w.n_probe, w.n_frames, w.ny, w.nx, seed=seed, dt_fs=w.dt_fs)
    tab = {k: torch.from_numpy(v).cuda() for k, v in X.tables().items()}
    return spec, tacaw.Producer(spec, tab)


def run(tacaw, w, prod, masks, batch):
    plan = w.plan(masks=torch.from_numpy(masks).cuda())
    assert plan.info()["tile_pixels"] == 32 and plan.info()["n_segments"] == 31
    buf = torch.empty((batch, w.push_frames or 200, w.ny, w.nx), dtype=torch.complex64,
                      device="cuda")
    for p0 in range(0, w.n_probe, batch):
        for f0 in range(0, w.n_frames, buf.shape[1]):
            prod.into(buf, probe0=p0, frame0=f0)
            plan.push(buf, probe0=p0)
    S = plan.finalize()
    D, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    info = plan.info()
    plan.close()
    return S.reshape(w.n_omega, -1), D.cpu().numpy(), Dp.cpu().numpy(), info


def check(w, spec, pix, masks, S, D, Dp, label):
    psi = X.generate(spec, pixels=pix)
    rows = axes.window_rows(w.seg_len, w.omega_half)
    So, Spo = O.tacaw_spectra_fft(psi, w.seg_len, w.hop, O.window("hann", w.seg_len))
    So, Spo = So[rows], Spo[:, rows]
    Mo = masks.reshape(masks.shape[0], -1)[:, pix]
    Do = O.detector_spectra(So, Mo)
    Dpo = np.transpose(O.detector_spectra(Spo, Mo), (1, 0, 2))
    eS = rel(S[:, torch.from_numpy(pix).cuda()].cpu().numpy(), So)
    eD = max(rel(D[j], Do[j]) for j in range(len(Mo)))
    eDp = max(rel(Dp[j], Dpo[j]) for j in range(len(Mo)))
    print(f"{label}: {pix.size} sampled pixels, S {eS:.2e} D {eD:.2e} D_p {eDp:.2e}", flush=True)
    assert eS <= 1e-5 and eD <= 1e-5 and eDp <= 1e-5


def test_paper_plane_wave_full_grid(tacaw):
    w = W.PAPER_PLANE_WAVE.replace(push_frames=200)
    assert (w.n_omega, w.n_frames, w.ny) == (181, 3200, 383)
    nk = w.ny * w.nx
    rng = np.random.default_rng(11)
    starts = np.arange(0, nk, 32)
    pix = np.unique(np.minimum(starts + rng.integers(0, 32, size=starts.size), nk - 1))
    pix = np.unique(np.append(pix, nk - 1))  # the one-pixel last tile
    ind = np.zeros(nk)
    ind[pix] = 1.0
    # two detectors on the sampled pixels: weights and a disk of 60 mrad
    disk = detectors.circular(w.ny, w.nx, W.mrad_radius_px(60.0))
    masks = np.stack([rng.random(nk) * ind, disk.reshape(-1) * ind]).reshape(2, w.ny, w.nx)
    spec, prod = producer(tacaw, w, seed=7)
    S, D, Dp, info = run(tacaw, w, prod, masks, batch=1)
    assert info["frames_dropped"] == 0 and info["probes_complete"] == 1
    check(w, spec, pix, masks, S, D, Dp, "plane wave, 383^2, L = 200, 181 bins")


def test_paper_stem_scan_in_batches(tacaw):
    w = W.PAPER_STEM.replace(n_probe=8, max_probes_in_flight=4)
    assert (w.n_omega, w.push_frames, len(w.detectors)) == (191, 200, 4)
    full = w.masks()
    nk = w.ny * w.nx
    inside = np.flatnonzero(full.reshape(4, -1).sum(axis=0) > 0)
    rng = np.random.default_rng(12)
    pix = np.sort(rng.choice(inside, size=600, replace=False))
    ind = np.zeros(nk)
    ind[pix] = 1.0
    masks = (full.reshape(4, -1) * ind).reshape(full.shape)
    assert all(masks[j].sum() > 0 for j in range(4))  # every detector keeps sampled pixels
    spec, prod = producer(tacaw, w, seed=8)
    S, D, Dp, info = run(tacaw, w, prod, masks, batch=4)
    assert info["probes_complete"] == 8
    check(w, spec, pix, masks, S, D, Dp, "STEM scan, 8 probes in batches of 4, 191 bins")
