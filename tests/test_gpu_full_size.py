"""Parity at the full workload sizes, in the launch configuration bench.py times
(one whole-series push), on outputs the oracle computes pixel by pixel: S (global
and per-chunk mean) and the gradient at seeded sampled pixels (every probe, every frame), regenerated
bit-identically on the CPU; detector spectra through properties that hold at any
size (D equals a float64 reduction of the GPU's S; the probe mean of D_p is D)."""

import numpy as np
import pytest
import torch

import oracle as O
import tacaw_synth as T

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def resident(spec):
    psi = torch.empty((spec.n_probe, spec.n_frames, spec.ny, spec.nx), dtype=spec.torch_dtype,
                      device="cuda")
    for p in range(spec.n_probe):
        T.generate_into(spec, psi[p:p + 1], probes=[p], frame_chunk=256)
    torch.cuda.synchronize()
    return psi


def test_realistic_workload_64_probes_256sq():
    # 64 probes x 2048 frames x 256 x 256 complex64 (68.7 GB), L = 512, H = 256, 4 masks
    from paper_2607_02236_amd import tacaw

    spec = T.config_realistic()
    L, H = 512, 256
    psi = resident(spec)
    masks = torch.from_numpy(T.standard_masks(256, 256)).cuda()
    plan = tacaw.Plan(spec.n_probe, 256, 256, spec.n_frames, L, H, masks=masks)
    plan.push(psi)
    S = plan.finalize()
    D, Dp = plan.detector_spectra(per_probe=True)
    # the per-chunk mean on the same resident series
    pseg = tacaw.Plan(spec.n_probe, 256, 256, spec.n_frames, L, H, mean_mode="per_segment")
    pseg.push(psi)
    S_seg = pseg.finalize()
    torch.cuda.synchronize()
    pseg.close()
    del psi
    pix = np.sort(np.random.default_rng(8).choice(256 * 256, size=48, replace=False))
    sample = T.generate(spec, pixels=pix).numpy()
    So, _ = O.tacaw_spectra_fft(sample, L, H, O.window("hann", L))
    Sso, _ = O.tacaw_spectra_fft(sample, L, H, O.window("hann", L), "per_segment")
    es = rel(S_seg.reshape(L, -1)[:, torch.from_numpy(pix).cuda()].cpu().numpy(), Sso)
    print(f"64 probes 256^2, per-chunk mean: S(sampled) {es:.2e}", flush=True)
    assert es <= 1e-5
    e = rel(S.reshape(L, -1)[:, torch.from_numpy(pix).cuda()].cpu().numpy(), So)
    Dref = torch.einsum("jk,mk->jm", masks.reshape(4, -1), S.reshape(L, -1))
    eD = max(rel(D[j].cpu(), Dref[j].cpu()) for j in range(4))
    eDp = rel(Dp.mean(dim=1).cpu(), D.cpu())
    print(f"64 probes 256^2: S(sampled) {e:.2e} D {eD:.2e} mean(Dp) {eDp:.2e}", flush=True)
    assert e <= 1e-5 and eD <= 1e-12 and eDp <= 1e-12
    plan.close()


def test_gradient_workload_16_probes_128sq():
    # 16 probes x 1024 frames x 128 x 128 complex64, L = 512, H = 512, 4 masks, loss
    # sum_j sum_m a_j(m) D_j(m): the gradient at pixel k needs only that pixel's series
    from paper_2607_02236_amd import autograd as ag

    spec = T.config_gradient()
    L, H = 512, 512
    psi = resident(spec)
    masks_np = T.standard_masks(128, 128, scale=0.5)
    a = T.loss_weights(4, L, seed=4)
    x = psi.requires_grad_(True)
    _, D, _ = ag.spectra(x, L, H, masks=torch.from_numpy(masks_np), window="hann_width",
                         window_param=1.0)
    (D * torch.from_numpy(a).cuda()).sum().backward()
    pix = np.sort(np.random.default_rng(9).choice(128 * 128, size=32, replace=False))
    g = x.grad.reshape(spec.n_probe, spec.n_frames, -1)[:, :, torch.from_numpy(pix).cuda()]
    g = g.cpu().numpy()
    gS = np.einsum("jm,jk->mk", a, masks_np.reshape(4, -1)[:, pix])
    g_o, _, _ = O.spectra_vjp(T.generate(spec, pixels=pix).numpy(), L, H,
                            O.window("hann_width", L, 1.0), gS)
    e = rel(g, g_o)
    print(f"gradient 16 probes 128^2: rel err (sampled pixels) {e:.2e}", flush=True)
    assert e <= 1e-5
