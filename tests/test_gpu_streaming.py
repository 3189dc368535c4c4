"""Streaming ingest at the large workload's real k-grid: 1024 x 1024 pixels,
L = 1024 with 50 % overlap, 4096 frames per probe pushed in chunks of 256 frames
that are generated on the GPU just before each push (the series is never held
whole), probes in batches through the plan's frame ring. S is checked against
the FP64 oracle on seeded sampled pixels (regenerated bit-identically on the
CPU); the detector spectra against a float64 torch reduction of the GPU's S."""

import numpy as np
import pytest
import torch

import oracle as O
import tacaw_synth as T

pytestmark = pytest.mark.gpu


def rel(a, b):
    # relative L2 error; absolute where the reference is exactly zero (a mask that
    # misses the sampled band gives D_j = 0 on both sides)
    nb = float(np.linalg.norm(np.asarray(b)))
    d = float(np.linalg.norm(np.asarray(a) - np.asarray(b)))
    return d / nb if nb > 0 else d


@pytest.mark.parametrize("n_probe,batch,grid,chunk,ring,tiled", [
    (4, 2, 256, 256, 0, False),        # quick: 256 x 256 grid
    (16, 4, 1024, 256, 0, False),      # one GPU's share of the 256-probe scan at the full grid
    (16, 4, 1024, 256, 2048, False),   # the same, deferred: chunks wait in a 2048-frame ring
    (16, 4, 1024, 256, 2048, True),    # the same with the ring stored per pixel tile
])
def test_streaming_pushes_match_oracle(n_probe, batch, grid, chunk, ring, tiled):
    from paper_2607_02236_amd import tacaw

    spec = T.config_streaming(n_probe=n_probe, n_frames=4096, ny=grid, nx=grid)
    L, H = 1024, 512
    # one sampled pixel in every 8-pixel tile of the chunk kernel on a band of 8
    # pixel rows through the centre; the masks are the standard ones restricted to
    # those pixels, so the oracle can reduce D and D_p itself
    rng = np.random.default_rng(5)
    rows = np.arange(grid // 2 - 4, grid // 2 + 4)
    pix = np.sort(np.concatenate([r * grid + np.arange(0, grid, 8) for r in rows])
                  + rng.integers(0, 8, size=rows.size * (grid // 8)))
    ind = np.zeros(grid * grid)
    ind[pix] = 1.0
    masks_np = T.standard_masks(grid, grid, scale=grid / 256).reshape(4, -1) * ind[None, :]
    masks = torch.from_numpy(masks_np.reshape(4, grid, grid)).cuda()
    plan = tacaw.Plan(n_probe, grid, grid, spec.n_frames, L, H, masks=masks,
                      max_probes_in_flight=batch, ring_frames=ring, tiled_ring=tiled)
    assert plan.info()["tile_pixels"] == 8
    buf = torch.empty((batch, chunk, grid, grid), dtype=torch.complex64, device="cuda")
    for p0 in range(0, n_probe, batch):
        for f0 in range(0, spec.n_frames, chunk):
            for i in range(batch):
                buf[i] = T.generate(spec, [p0 + i], (f0, f0 + chunk), device="cuda")[0]
            plan.push(buf, probe0=p0)
        print(f"probes {p0}..{p0 + batch - 1} pushed", flush=True)
    S = plan.finalize()
    D, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    info = plan.info()
    assert info["n_segments"] == 7 and info["probes_complete"] == n_probe

    print(f"regenerating {pix.size} sampled pixels on the CPU", flush=True)
    psi = T.generate(spec, pixels=pix).numpy()
    So, Spo = O.tacaw_spectra_fft(psi, L, H, O.window("hann", L))
    del psi
    Sg = S.reshape(L, -1)[:, torch.from_numpy(pix).cuda()].cpu().numpy()
    e = rel(Sg, So)
    Dref = torch.einsum("jk,mk->jm", masks.reshape(masks.shape[0], -1), S.reshape(L, -1))
    eD = max(rel(D[j].cpu(), Dref[j].cpu()) for j in range(D.shape[0]))
    eDp = rel(Dp.mean(dim=1).cpu(), D.cpu())  # probe mean of per-probe spectra = D
    print(f"streaming {n_probe} probes {grid}^2 ring {ring}{' tiled' if tiled else ''}: "
          f"S(sampled) {e:.2e} D {eD:.2e} "
          f"mean(Dp) {eDp:.2e}")
    assert e <= 1e-5 and eD <= 1e-12 and eDp <= 1e-12
    Mo = masks_np[:, pix]
    Do = O.detector_spectra(So, Mo)
    Dpo = np.transpose(O.detector_spectra(Spo, Mo), (1, 0, 2))
    eDo = max(rel(D[j].cpu().numpy(), Do[j]) for j in range(4))
    eDpo = max(rel(Dp[j].cpu().numpy(), Dpo[j]) for j in range(4))
    print(f"  sampled-pixel detectors vs oracle: D {eDo:.2e} D_p {eDpo:.2e}", flush=True)
    assert eDo <= 1e-5 and eDpo <= 1e-5
    plan.close()


def test_zero_copy_ingest_generator_writes_into_ring():
    # the seeded generator (the producer) writes each piece straight into the
    # plan's ring; results equal pushing the same series, and the oracle
    from paper_2607_02236_amd import tacaw

    spec = T.SeriesSpec(3, 640, 10, 12, dtype="c64", seed=71, model="lines", n_terms=8)
    L, H, D, piece = 128, 64, 256, 64
    masks = torch.from_numpy(T.standard_masks(10, 12, scale=0.06)).cuda()
    psi = T.generate(spec)
    ref = tacaw.Plan(3, 10, 12, 640, L, H, masks=masks)
    ref.push(psi.cuda())
    S_ref = ref.finalize()
    _, Dp_ref = ref.detector_spectra(per_probe=True)
    plan = tacaw.Plan(3, 10, 12, 640, L, H, masks=masks, ring_frames=D, max_probes_in_flight=2)
    for p0, n in ((0, 2), (2, 1)):
        for f0 in range(0, 640, piece):
            view = plan.ingest(piece, probe0=p0, n_probes=n)
            for i in range(n):
                view[i] = T.generate(spec, [p0 + i], (f0, f0 + piece), device="cuda")[0]
            plan.commit()
    S = plan.finalize()
    _, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    assert rel(S.cpu(), S_ref.cpu()) < 1e-12 and rel(Dp.cpu(), Dp_ref.cpu()) < 1e-12
    So, _ = O.tacaw_spectra(psi.numpy(), L, H, O.window("hann", L))
    e = rel(S.cpu().numpy().reshape(L, -1), So)
    print(f"zero-copy ingest: S {e:.2e}")
    assert e <= 1e-5
    ref.close()
    plan.close()


def test_zero_copy_ingest_errors():
    from paper_2607_02236_amd import tacaw

    imm = tacaw.Plan(1, 4, 4, 512, 128, 64)
    with pytest.raises(tacaw.TacawError) as e:
        imm.ingest(64)
    assert e.value.kind == "STATE"
    imm.close()
    plan = tacaw.Plan(2, 4, 4, 512, 128, 64, ring_frames=256)
    with pytest.raises(tacaw.TacawError) as e:
        plan.ingest(129)  # more than ring_frames - seg_len
    assert e.value.kind == "SHAPE"
    v = plan.ingest(96, n_probes=2)
    v.fill_(1.0)
    with pytest.raises(tacaw.TacawError) as e:
        plan.push(torch.ones((2, 8, 4, 4), dtype=torch.complex64, device="cuda"))
    assert e.value.kind == "STATE"  # an ingest is open
    plan.commit()
    with pytest.raises(tacaw.TacawError) as e:
        plan.ingest(128, n_probes=2)  # rows 96..223 fit; 96 + 128 = 224 <= 256 is fine
        plan.commit()
        plan.ingest(64, n_probes=2)   # rows 224..287 would wrap
    assert e.value.kind == "SHAPE"
    plan.close()
