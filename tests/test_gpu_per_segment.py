"""Per-chunk mean (mean_mode="per_segment", scipy's detrend='constant'): each Welch
chunk subtracts the unweighted mean of its own L frames before the window.

The chunk kernel transforms psi - c (c = frame 0) as in the global mode; an FP64
pass over the pushed frames keeps each open chunk's sums and corrects the bins
where the window's DFT is non-zero. Checked against the FP64 oracle (itself
pinned to scipy.signal.welch for this mode) on seeded inputs, across hops that
let one frame fall in 1 to 4 chunks, ragged tails, streamed pushes, both ring
layouts, zero-copy ingest, an energy window and complex128 input."""

import numpy as np
import pytest
import torch

import oracle as O
import tacaw_synth as T

pytestmark = pytest.mark.gpu


def rel(a, b):
    # relative L2 error; absolute where the reference is exactly zero (a mask
    # that misses a tiny grid gives D_j = 0 on both sides)
    a = np.asarray(a)
    b = np.asarray(b)
    nb = float(np.linalg.norm(b.ravel()))
    d = float(np.linalg.norm((a - b).ravel()))
    return d / nb if nb > 0 else d


@pytest.fixture(scope="module")
def tacaw():
    from paper_2607_02236_amd import tacaw as t

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return t


def series(P, NT, ny, nx, seed, dtype="c64"):
    spec = T.SeriesSpec(P, NT, ny, nx, dtype=dtype, seed=seed, model="lines", n_terms=8,
                        amplitude=1e-3 / np.sqrt(8))
    return T.generate(spec)


def masks_for(ny, nx, seed):
    m = T.standard_masks(ny, nx, scale=min(ny, nx) / 128)
    m[3] = np.random.default_rng(seed).random((ny, nx))
    return m


def run(tacaw, psi, L, H, masks, pieces=None, **kw):
    P, NT, ny, nx = psi.shape
    plan = tacaw.Plan(P, ny, nx, NT, L, H, masks=torch.from_numpy(masks).cuda(), **kw)
    x = psi.cuda()
    if pieces is None:
        plan.push(x)
    else:
        f0 = 0
        for n in pieces:
            plan.push(x[:, f0:f0 + n])
            f0 += n
        assert f0 == NT
    S = plan.finalize()
    D, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    out = {"S": S.cpu().numpy().reshape(plan.n_omega, -1), "D": D.cpu().numpy(),
           "Dp": Dp.cpu().numpy()}
    plan.close()
    return out


def oracle(psi, L, H, masks, window="hann", rows=None):
    S, Sp = O.tacaw_spectra(psi.numpy(), L, H, O.window(window, L), "per_segment")
    if rows is not None:
        S, Sp = S[rows], Sp[:, rows]
    return {"S": S, "D": O.detector_spectra(S, masks),
            "Dp": np.transpose(O.detector_spectra(Sp, masks), (1, 0, 2))}


def check(g, o, tol, label):
    eS = rel(g["S"], o["S"])
    eD = max(rel(g["D"][j], o["D"][j]) for j in range(o["D"].shape[0]))
    eDp = max(rel(g["Dp"][j], o["Dp"][j]) for j in range(o["D"].shape[0]))
    print(f"{label}: S {eS:.2e} D {eD:.2e} Dp {eDp:.2e}", flush=True)
    assert eS <= tol and eD <= tol and eDp <= tol


@pytest.mark.parametrize("L,H,NT,ny,nx,P,window", [
    (128, 64, 1000, 7, 9, 3, "hann"),     # 2 chunks per frame, ragged tail
    (256, 256, 700, 5, 6, 2, "hann"),     # hop = L: 1 chunk per frame
    (512, 256, 2048, 4, 16, 2, "hann"),   # the large workload's chunk shape
    (200, 100, 3200, 3, 5, 1, "hann"),    # L = 200, 15 fs: 31 chunks
    (128, 32, 600, 4, 4, 2, "hann"),      # hop = L/4: 4 chunks per frame
    (64, 48, 500, 3, 3, 1, "hann"),       # hop that does not divide L
    (128, 64, 700, 4, 5, 2, "rect"),      # the window's DFT lives on bin 0 only
    (1024, 512, 2600, 3, 7, 1, "hann"),
])
def test_per_segment_matches_oracle(tacaw, L, H, NT, ny, nx, P, window):
    psi = series(P, NT, ny, nx, seed=L + H + NT)
    masks = masks_for(ny, nx, 5)
    g = run(tacaw, psi, L, H, masks, mean_mode="per_segment", window=window)
    check(g, oracle(psi, L, H, masks, window), 1e-5, f"per-chunk mean L={L} H={H} {window}")


def test_only_the_correction_bins_differ_from_the_global_mode(tacaw):
    # same chunk kernel arithmetic: every row but bins 0, +-1 is bit-identical
    L, H, NT, ny, nx, P = 256, 128, 900, 6, 8, 2
    psi = series(P, NT, ny, nx, seed=41)
    masks = masks_for(ny, nx, 6)
    g = run(tacaw, psi, L, H, masks, mean_mode="global")
    s = run(tacaw, psi, L, H, masks, mean_mode="per_segment")
    other = np.setdiff1d(np.arange(L), [0, 1, L - 1])
    assert np.array_equal(g["S"][other], s["S"][other])
    assert np.array_equal(g["Dp"][:, :, other], s["Dp"][:, :, other])
    assert not np.array_equal(g["S"][0], s["S"][0])


def test_static_wave_gives_exactly_zero(tacaw):
    # a time-independent wave: every chunk equals its own mean, S and D are 0
    L, H, NT, ny, nx = 128, 64, 500, 5, 7
    rng = np.random.default_rng(3)
    frame = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    psi = torch.from_numpy(np.broadcast_to(frame, (2, NT, ny, nx)).copy())
    g = run(tacaw, psi, L, H, masks_for(ny, nx, 7), mean_mode="per_segment")
    assert np.all(g["S"] == 0.0) and np.all(g["D"] == 0.0) and np.all(g["Dp"] == 0.0)


@pytest.mark.parametrize("pieces", [[1, 36, 100, 5, 258, 600], [128] * 7 + [104], [999, 1]])
def test_streamed_pushes_equal_one_push(tacaw, pieces):
    L, H, NT, ny, nx, P = 128, 64, 1000, 6, 5, 2
    psi = series(P, NT, ny, nx, seed=17)
    masks = masks_for(ny, nx, 8)
    whole = run(tacaw, psi, L, H, masks, mean_mode="per_segment")
    part = run(tacaw, psi, L, H, masks, pieces=pieces, mean_mode="per_segment")
    for key in ("S", "D", "Dp"):
        assert rel(part[key], whole[key]) <= 1e-12, key
    check(part, oracle(psi, L, H, masks), 1e-5, f"per-chunk mean, pushes {pieces[:3]}...")


@pytest.mark.parametrize("tiled", [False, True])
def test_deferred_ring_layouts(tacaw, tiled):
    L, H, NT, ny, nx, P = 256, 128, 1100, 9, 11, 2
    psi = series(P, NT, ny, nx, seed=23)
    masks = masks_for(ny, nx, 9)
    pieces = [128] * 8 + [76]
    g = run(tacaw, psi, L, H, masks, pieces=pieces, mean_mode="per_segment", ring_frames=512,
            tiled_ring=tiled)
    check(g, oracle(psi, L, H, masks), 1e-5, f"per-chunk mean, deferred ring tiled={tiled}")


def test_zero_copy_ingest(tacaw):
    spec = T.SeriesSpec(3, 640, 10, 12, dtype="c64", seed=72, model="lines", n_terms=8)
    L, H, D, piece = 128, 64, 256, 64
    masks = T.standard_masks(10, 12, scale=0.06)
    psi = T.generate(spec)
    plan = tacaw.Plan(3, 10, 12, 640, L, H, masks=torch.from_numpy(masks).cuda(), ring_frames=D,
                      max_probes_in_flight=2, mean_mode="per_segment")
    for p0, n in ((0, 2), (2, 1)):
        for f0 in range(0, 640, piece):
            view = plan.ingest(piece, probe0=p0, n_probes=n)
            for i in range(n):
                view[i] = T.generate(spec, [p0 + i], (f0, f0 + piece), device="cuda")[0]
            plan.commit()
    S = plan.finalize()
    Dv, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    g = {"S": S.cpu().numpy().reshape(L, -1), "D": Dv.cpu().numpy(), "Dp": Dp.cpu().numpy()}
    plan.close()
    check(g, oracle(psi, L, H, masks), 1e-5, "per-chunk mean, zero-copy ingest")


def test_energy_window_and_complex128(tacaw):
    L, H, NT, ny, nx, P, M = 256, 128, 800, 5, 9, 2, 40
    psi = series(P, NT, ny, nx, seed=57, dtype="c128")
    masks = masks_for(ny, nx, 10)
    g = run(tacaw, psi, L, H, masks, mean_mode="per_segment", in_dtype="c128", omega_half=M)
    rows = np.mod(np.arange(-M, M + 1), L)
    check(g, oracle(psi, L, H, masks, rows=rows), 1e-5, "per-chunk mean, window + c128")


def test_per_segment_refusals(tacaw):
    with pytest.raises(tacaw.TacawError) as e:  # Tukey's DFT is not confined to bins 0, +-1
        tacaw.Plan(1, 4, 4, 256, 128, 64, window="tukey", window_param=0.3,
                   mean_mode="per_segment")
    assert e.value.kind == "UNSUPPORTED"
    with pytest.raises(tacaw.TacawError) as e:  # fp16 GEMM scales from the whole series
        tacaw.Plan(1, 4, 4, 256, 128, 64, transform="gemm_f16x3", mean_mode="per_segment")
    assert e.value.kind == "UNSUPPORTED"


@pytest.mark.parametrize("L,H,NT,ny,nx,P,dtype,window", [
    (256, 128, 900, 9, 13, 2, "c64", "hann"),        # hop = L/2, ragged tail
    (512, 512, 1100, 5, 17, 2, "c64", "hann_width"),  # hop = L, width-r Hann (r = 1)
    (128, 64, 700, 6, 7, 3, "c128", "hann"),
    (512, 256, 1600, 4, 16, 1, "c64", "rect"),       # W(m) != 0 at bin 0 only
    (1024, 512, 2600, 3, 5, 1, "c64", "hann"),
])
def test_per_segment_adjoint_matches_oracle(tacaw, L, H, NT, ny, nx, P, dtype, window):
    # loss = <a, D> + <b, D_p> + <gS, S>: each chunk's own mean is part of the
    # differentiated map, so frames of chunk s carry 2 w g_s - M_s / L
    from paper_2607_02236_amd import autograd as ag

    psi = series(P, NT, ny, nx, seed=L + NT + P, dtype=dtype)
    masks = T.standard_masks(ny, nx, scale=min(ny, nx) / 64)
    rng = np.random.default_rng(L + H)
    a = rng.random((4, L))
    b = rng.random((4, P, L)) * 0.3
    gS = rng.random((L, ny * nx)) * 0.1
    x = psi.cuda().requires_grad_(True)
    S, D, Dp = ag.spectra(x, L, H, masks=torch.from_numpy(masks), window=window,
                          mean_mode="per_segment")
    loss = (D * torch.from_numpy(a).cuda()).sum() + (Dp * torch.from_numpy(b).cuda()).sum() \
        + (S.reshape(L, -1) * torch.from_numpy(gS).cuda()).sum()
    loss.backward()
    Mf = masks.reshape(4, -1)
    gS_full = gS + np.einsum("jm,jk->mk", a, Mf)
    gSp_full = np.einsum("jpm,jk->pmk", b, Mf)
    w = O.window(window, L, 1.0) if window == "hann_width" else O.window(window, L)
    g_o, _, lval = O.spectra_vjp(psi.numpy(), L, H, w, gS_full, gSp_full, mean_mode="per_segment")
    assert float(loss) == pytest.approx(lval, rel=1e-5)
    e = rel(x.grad.cpu().numpy().reshape(g_o.shape), g_o)
    print(f"per-chunk mean adjoint L={L} H={H} {dtype} {window}: grad {e:.2e}", flush=True)
    assert e <= 1e-5
