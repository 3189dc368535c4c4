"""Degenerate shapes against the FP64 oracle: a single pixel (one valid lane in a
tile), a series exactly one chunk long, a hop of one frame (every frame starts a
chunk), and a push of zero frames through the C ABI (a no-op); and non-finite
exit waves, which the optional finite check reports at finalize."""

import ctypes

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


@pytest.mark.parametrize("L,H,NT,ny,nx,P,dtype", [
    (64, 32, 64, 1, 1, 1, "c64"),       # one pixel, one chunk
    (512, 256, 1000, 1, 1, 2, "c64"),   # one pixel, several probes
    (1024, 512, 1024, 3, 3, 1, "c128"),  # exactly one chunk at the longest L
    (128, 1, 200, 2, 3, 1, "c64"),      # hop 1: 73 chunks, each frame starts one
    (200, 100, 200, 1, 1, 1, "c64"),    # L = 200, one chunk, one pixel
])
def test_degenerate_shapes_match_oracle(L, H, NT, ny, nx, P, dtype):
    from paper_2607_02236_amd import tacaw

    spec = T.SeriesSpec(P, NT, ny, nx, dtype=dtype, seed=L + H + NT, model="lines", n_terms=8,
                        amplitude=1e-3 / np.sqrt(8))
    psi = T.generate(spec)
    ones = np.ones((1, ny, nx))
    plan = tacaw.Plan(P, ny, nx, NT, L, H, in_dtype=dtype, masks=torch.from_numpy(ones).cuda())
    plan.push(psi.cuda())
    S = plan.finalize().cpu().numpy().reshape(L, -1)
    D, Dp = plan.detector_spectra(per_probe=True)
    info = plan.info()
    plan.close()
    So, Spo = O.tacaw_spectra(psi.numpy(), L, H, O.window("hann", L))
    assert info["n_segments"] == O.segment_count(NT, L, H)
    eS = rel(S, So)
    eD = rel(D.cpu().numpy()[0], So.sum(axis=1))  # a mask of ones sums S over pixels
    eDp = rel(Dp.cpu().numpy()[0], Spo.sum(axis=2))
    print(f"L={L} H={H} NT={NT} {ny}x{nx} P={P} {dtype}: S {eS:.2e} D {eD:.2e} Dp {eDp:.2e}",
          flush=True)
    assert eS <= 1e-5 and eD <= 1e-5 and eDp <= 1e-5


def test_zero_frame_push_is_a_no_op():
    from paper_2607_02236_amd import tacaw

    spec = T.SeriesSpec(2, 300, 4, 5, dtype="c64", seed=5, model="lines", n_terms=8)
    psi = T.generate(spec).cuda()
    ref = tacaw.Plan(2, 4, 5, 300, 128, 64)
    ref.push(psi)
    S_ref = ref.finalize().cpu()
    ref.close()
    plan = tacaw.Plan(2, 4, 5, 300, 128, 64)
    plan.push(psi[:, :100])
    rc = tacaw.lib.tacaw_push_frames(plan.handle, ctypes.c_void_p(psi.data_ptr()), 0, 2, 0,
                                     psi.stride(0), psi.stride(1))
    assert rc == 0
    plan.push(psi[:, 100:])
    S = plan.finalize().cpu()
    plan.close()
    assert torch.equal(S, S_ref)


def test_nonfinite_input_is_reported_with_the_check_flag():
    # a NaN and an Inf exit wave propagate into their pixels' spectra; with
    # check_finite the finalize reports them (NONFINITE, plan finalized, count in
    # info); without it nothing checks; clean input passes the check
    from paper_2607_02236_amd import tacaw

    L, H, NT, ny, nx, P = 128, 64, 320, 3, 4, 2
    spec = T.SeriesSpec(P, NT, ny, nx, dtype="c64", seed=17, model="lines", n_terms=4)
    clean = T.generate(spec).cuda()
    bad = clean.clone()
    bad[0, 100, 1, 2] = complex(float("nan"), 0.0)
    bad[1, 7, 2, 0] = complex(float("inf"), 1.0)
    masks = torch.from_numpy(T.standard_masks(ny, nx, scale=0.1)).cuda()

    plan = tacaw.Plan(P, ny, nx, NT, L, H, masks=masks, check_finite=True)
    plan.push(clean)
    S = plan.finalize()
    assert plan.info()["nonfinite"] == 0 and torch.isfinite(S).all()
    plan.close()

    plan = tacaw.Plan(P, ny, nx, NT, L, H, masks=masks, check_finite=True)
    plan.push(bad)
    with pytest.raises(tacaw.TacawError) as e:
        plan.finalize()
    assert e.value.kind == "NONFINITE"
    S = e.value.result
    n = plan.info()["nonfinite"]
    bad_S = int((~torch.isfinite(S)).sum())
    print(f"non-finite values reported {n}, in S {bad_S}", flush=True)
    assert plan.info()["state"] == 1 and n >= bad_S > 0
    # only the two poisoned pixels' columns of S are affected
    cols = (~torch.isfinite(S)).reshape(L, -1).any(dim=0).nonzero().flatten().tolist()
    assert cols == sorted([1 * nx + 2, 2 * nx + 0])
    D, Dp = plan.detector_spectra(per_probe=True)  # the plan is usable after the report
    plan.close()

    plan = tacaw.Plan(P, ny, nx, NT, L, H, masks=masks)
    plan.push(bad)
    S = plan.finalize()  # no check: the NaN propagates silently
    assert not torch.isfinite(S).all() and plan.info()["nonfinite"] == 0
    plan.close()
