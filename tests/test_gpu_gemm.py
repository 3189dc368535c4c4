"""DFT-as-GEMM form (MFMA, split-precision operands) against the FP64 oracle and
the FP32 FFT form, per detector spectrum."""

import numpy as np
import pytest
import torch

import oracle as O
import tacaw_synth as T

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def tacaw():
    from paper_2607_02236_amd import tacaw as t

    assert torch.cuda.is_available()
    return t


def run(tacaw, psi, L, H, masks, transform, **kw):
    P, NT, ny, nx = psi.shape
    in_dtype = "c64" if psi.dtype == torch.complex64 else "c128"
    plan = tacaw.Plan(P, ny, nx, NT, L, H, in_dtype=in_dtype, transform=transform,
                      masks=torch.from_numpy(masks).cuda(), **kw)
    plan.push(psi.cuda())
    S = plan.finalize().cpu().numpy().reshape(L, -1)
    D, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    out = S, D.cpu().numpy(), Dp.cpu().numpy()
    plan.close()
    return out


# bars: FP16 x3 (22 significant bits) meets the FP32-FFT bar; BF16 x3 keeps
# about 16 bits, so its error is reported against a looser bound
BARS = {"gemm_f16x3": 1e-5, "gemm_bf16x3": 1e-4}


@pytest.mark.parametrize("nt", [512, 256])
@pytest.mark.parametrize("form", ["gemm_f16x3", "gemm_bf16x3"])
def test_precision_form_single_chunk(tacaw, nt, form):
    # 1 probe, 64 x 64, complex128, one Hann chunk of N_t = L frames
    spec = T.config_precision(n_frames=nt)
    psi = T.generate(spec)
    masks = np.stack([T.disk_mask(64, 64, 24, inner=8), T.standard_masks(64, 64, 0.25)[0]])
    S, D, Dp = run(tacaw, psi, nt, nt, masks, form)
    So, _ = O.tacaw_spectra(psi.numpy(), nt, nt, O.window("hann", nt))
    Do = O.detector_spectra(So, masks)
    Sf, Df, _ = run(tacaw, psi, nt, nt, masks, "fft")
    eS = rel(S, So)
    eD = [rel(D[j], Do[j]) for j in range(2)]
    eF = [rel(D[j], Df[j]) for j in range(2)]
    eFo = [rel(Df[j], Do[j]) for j in range(2)]
    print(f"{form} N_t=L={nt}: S {eS:.2e} D vs oracle {eD[0]:.2e} {eD[1]:.2e} "
          f"D vs FFT {eF[0]:.2e} {eF[1]:.2e} FFT vs oracle {eFo[0]:.2e} {eFo[1]:.2e}")
    assert eS <= BARS[form] and max(eD) <= BARS[form]
    np.testing.assert_allclose(Dp[:, 0, :], D, rtol=1e-12, atol=0)  # one probe


@pytest.mark.parametrize("form", ["gemm_f16x3", "gemm_bf16x3"])
@pytest.mark.parametrize("L,H,NT,ny,nx,P", [
    (128, 64, 640, 9, 11, 3),
    (256, 256, 768, 12, 12, 2),
    (512, 256, 1024, 8, 9, 2),
])
def test_gemm_multi_probe_multi_chunk(tacaw, form, L, H, NT, ny, nx, P):
    spec = T.SeriesSpec(P, NT, ny, nx, dtype="c64", seed=L + 7, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(ny, nx, scale=min(ny, nx) / 128)
    masks[3] = np.random.default_rng(3).random((ny, nx))
    S, D, Dp = run(tacaw, psi, L, H, masks, form)
    So, Spo = O.tacaw_spectra(psi.numpy(), L, H, O.window("hann", L))
    Do = O.detector_spectra(So, masks)
    Dpo = np.transpose(O.detector_spectra(Spo, masks), (1, 0, 2))
    e = max([rel(S, So)] + [rel(D[j], Do[j]) for j in range(4)] + [rel(Dp[j], Dpo[j]) for j in range(4)])
    print(f"{form} L={L} H={H} P={P}: max rel err {e:.2e}")
    assert e <= BARS[form]


@pytest.mark.parametrize("form,roi", [("gemm_bf16x3", 0), ("gemm_f16x3", 0), ("gemm_bf16x3", 100.0)])
def test_gemm_chunk_length_1024(tacaw, form, roi):
    # L = 1024: all bins need two row groups of the GEMM; an energy window one
    from paper_2607_02236_amd import axes

    L, H, NT, ny, nx, P = 1024, 512, 2048, 6, 11, 2
    spec = T.SeriesSpec(P, NT, ny, nx, dtype="c64", seed=97, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(ny, nx, scale=min(ny, nx) / 128)
    masks[3] = np.random.default_rng(4).random((ny, nx))
    M = axes.omega_half_for(L, 5.0, e_max_mev=roi) if roi else 0
    plan = tacaw.Plan(P, ny, nx, NT, L, H, transform=form, masks=torch.from_numpy(masks).cuda(),
                      omega_half=M)
    plan.push(psi.cuda())
    S = plan.finalize().cpu().numpy().reshape(plan.n_omega, -1)
    D, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    So, Spo = O.tacaw_spectra(psi.numpy(), L, H, O.window("hann", L))
    rows = (np.arange(plan.n_omega) - M) % L if M else np.arange(L)
    So, Spo = So[rows], Spo[:, rows]
    Do = O.detector_spectra(So, masks)
    Dpo = np.transpose(O.detector_spectra(Spo, masks), (1, 0, 2))
    e = max([rel(S, So)] + [rel(D.cpu().numpy()[j], Do[j]) for j in range(4)]
            + [rel(Dp.cpu().numpy()[j], Dpo[j]) for j in range(4)])
    print(f"{form} L=1024 window {roi} meV ({plan.n_omega} bins): max rel err {e:.2e}")
    assert e <= BARS[form]
    plan.close()


@pytest.mark.parametrize("ring,tiled,dtype", [(0, False, "c64"), (2048, False, "c64"),
                                              (2048, True, "c64"), (0, False, "c128")])
def test_gemm_bf16_streamed_pushes(tacaw, ring, tiled, dtype):
    # the streaming form: a reference fixed by the first chunk and the exact FP64
    # mean correction, frames before a push from the ring (immediate, deferred, tiled)
    L, H, NT, ny, nx, P, piece = 1024, 512, 3072, 5, 13, 2, 256
    spec = T.SeriesSpec(P, NT, ny, nx, dtype=dtype, seed=98, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(ny, nx, scale=min(ny, nx) / 128)
    masks[3] = np.random.default_rng(5).random((ny, nx))
    plan = tacaw.Plan(P, ny, nx, NT, L, H, transform="gemm_bf16x3", in_dtype=dtype,
                      masks=torch.from_numpy(masks).cuda(), ring_frames=ring, tiled_ring=tiled)
    x = psi.cuda()
    for f0 in range(0, NT, piece):
        plan.push(x[:, f0:f0 + piece])
    S = plan.finalize().cpu().numpy().reshape(L, -1)
    D, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    So, Spo = O.tacaw_spectra(psi.numpy(), L, H, O.window("hann", L))
    Do = O.detector_spectra(So, masks)
    Dpo = np.transpose(O.detector_spectra(Spo, masks), (1, 0, 2))
    e = max([rel(S, So)] + [rel(D.cpu().numpy()[j], Do[j]) for j in range(4)]
            + [rel(Dp.cpu().numpy()[j], Dpo[j]) for j in range(4)])
    rows = [0, 1, L - 1]
    eR = rel(S[rows], So[rows])
    print(f"bf16x3 streamed {dtype} (ring {ring}{' tiled' if tiled else ''}): max rel err {e:.2e}, "
          f"rows 0, +-1 {eR:.2e}")
    assert e <= BARS["gemm_bf16x3"] and eR <= BARS["gemm_bf16x3"]
    plan.close()


@pytest.mark.parametrize("roi", [0, 60])
def test_gemm_bf16_per_chunk_mean(tacaw, roi):
    # per-chunk mean with the bf16 GEMM form: the FP64 per-chunk kernel supplies the
    # correction rows, the GEMM kernel every other row; streamed pushes
    L, H, NT, ny, nx, P, piece = 512, 256, 1536, 6, 7, 2, 192
    spec = T.SeriesSpec(P, NT, ny, nx, dtype="c64", seed=77, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(ny, nx, scale=min(ny, nx) / 128)
    from paper_2607_02236_amd import axes

    M = axes.omega_half_for(L, 5.0, e_max_mev=roi) if roi else 0
    plan = tacaw.Plan(P, ny, nx, NT, L, H, transform="gemm_bf16x3", mean_mode="per_segment",
                      masks=torch.from_numpy(masks).cuda(), dt_fs=5.0, omega_half=M)
    x = psi.cuda()
    for f0 in range(0, NT, piece):
        plan.push(x[:, f0:f0 + piece])
    S = plan.finalize().cpu().numpy().reshape(plan.n_omega, -1)
    D, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    So, Spo = O.tacaw_spectra(psi.numpy(), L, H, O.window("hann", L), "per_segment")
    rows = axes.window_rows(L, M)
    So, Spo = So[rows], Spo[:, rows]
    Do = O.detector_spectra(So, masks)
    Dpo = np.transpose(O.detector_spectra(Spo, masks), (1, 0, 2))
    e = max([rel(S, So)] + [rel(D.cpu().numpy()[j], Do[j]) for j in range(4)]
            + [rel(Dp.cpu().numpy()[j], Dpo[j]) for j in range(4)])
    corr = [int(np.flatnonzero(rows == b)[0]) for b in (0, 1, L - 1)]
    eR = rel(S[corr], So[corr])
    print(f"bf16x3 per-chunk mean (window {roi} meV, {plan.n_omega} bins): max rel err {e:.2e}, "
          f"rows 0, +-1 {eR:.2e}")
    assert e <= BARS["gemm_bf16x3"] and eR <= 1e-6
    plan.close()


def test_gemm_rejects_streaming_fp16_and_unsupported_lengths(tacaw):
    with pytest.raises(tacaw.TacawError) as e:
        tacaw.Plan(1, 4, 4, 400, 200, 100, transform="gemm_bf16x3")
    assert e.value.kind == "UNSUPPORTED"
    # fp16 scales its operands from the whole series: whole-series pushes only
    plan = tacaw.Plan(1, 4, 4, 512, 256, 128, transform="gemm_f16x3")
    psi = T.generate(T.SeriesSpec(1, 512, 4, 4)).cuda()
    with pytest.raises(tacaw.TacawError) as e:
        plan.push(psi[:, :300])
    assert e.value.kind == "UNSUPPORTED"
    plan.close()
