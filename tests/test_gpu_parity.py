"""GPU parity of the FFT path against the FP64 oracle (through the C ABI).

Inputs come from the seeded generator (tacaw_synth) and are handed bit-for-bit
to both sides. The bar for the FP32 FFT path: relative L2 error <= 1e-5 for S
(Frobenius) and for every detector spectrum D_j and per-probe D_{j,p}.
"""

import sys

import numpy as np
import pytest
import torch

import oracle as O
import tacaw_synth as T

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tacaw():
    from paper_2607_02236_amd import tacaw as t

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return t


def rel(a, b):
    # relative L2 error; complex arrays keep their imaginary parts
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def run_gpu(tacaw, psi, L, H, masks=None, pushes=None, probe_batches=None, **kw):
    """psi: CPU complex tensor [P, NT, ny, nx]; pushes: list of frame counts."""
    P, NT, ny, nx = psi.shape
    dev = psi.cuda()
    m = torch.from_numpy(masks).cuda() if masks is not None else None
    in_dtype = "c64" if psi.dtype == torch.complex64 else "c128"
    plan = tacaw.Plan(P, ny, nx, NT, L, H, in_dtype=in_dtype, masks=m, **kw)
    batches = probe_batches or [(0, P)]
    for p0, p1 in batches:
        f0 = 0
        for n in (pushes or [NT]):
            plan.push(dev[p0:p1, f0:f0 + n], probe0=p0)
            f0 += n
        assert f0 == NT
    S = plan.finalize()
    out = {"S": S.cpu().numpy().reshape(L, -1), "info": plan.info()}
    if masks is not None:
        D, Dp = plan.detector_spectra(per_probe=True)
        out["D"] = D.cpu().numpy()
        out["Dp"] = Dp.cpu().numpy()
    torch.cuda.synchronize()
    plan.close()
    return out


def oracle_all(psi, L, H, window="hann", param=None, masks=None, mean_mode="global",
               probe_reduce="mean", fft=False):
    w = O.window(window, L, param)
    S, Sp = O.tacaw_spectra(psi.numpy(), L, H, w, mean_mode, probe_reduce, fft=fft)
    out = {"S": S, "Sp": Sp}
    if masks is not None:
        out["D"] = O.detector_spectra(S, masks)
        out["Dp"] = np.transpose(O.detector_spectra(Sp, masks), (1, 0, 2))
    return out


def check(g, o, tol=TOL, label=""):
    eS = rel(g["S"], o["S"])
    msg = f"{label} S {eS:.2e}"
    assert eS <= tol, msg
    if "D" in o:
        for j in range(o["D"].shape[0]):
            eD = rel(g["D"][j], o["D"][j])
            eDp = rel(g["Dp"][j], o["Dp"][j])
            msg += f" D{j} {eD:.2e} Dp{j} {eDp:.2e}"
            assert eD <= tol and eDp <= tol, msg
    say(msg)


def test_plain_one_probe_complex128(tacaw):
    # 1 probe, 256 frames at 5 fs, 64 x 64, complex128, one Hann chunk, one annulus
    spec = T.config_plain_1probe()
    psi = T.generate(spec)
    masks = T.disk_mask(64, 64, 24, inner=8)[None]
    g = run_gpu(tacaw, psi, 256, 256, masks)
    o = oracle_all(psi, 256, 256, masks=masks)
    check(g, o, label="plain c128 L=256")
    assert g["info"]["n_segments"] == 1


@pytest.mark.parametrize("L,H,NT,ny,nx,P", [
    (64, 32, 200, 7, 9, 2),        # ragged pixels (63), tail frames dropped
    (128, 64, 640, 37, 29, 3),     # ragged 1073 pixels, 9 chunks
    (256, 128, 700, 16, 20, 2),
    (512, 256, 1536, 12, 25, 2),   # N1 = 32 kernel
    (512, 512, 1100, 9, 9, 1),     # no overlap, dropped tail
    (1024, 512, 2048, 5, 20, 1),
    (256, 100, 900, 11, 11, 2),    # hop not dividing L: chunk reload path
    (200, 100, 3200, 6, 7, 1),     # Sec. III.A worked example: L = 200, nu = 2, 31 chunks
    (200, 100, 700, 9, 13, 2),     # prime-factor 10-point passes, ragged tiles of 32
    (200, 200, 650, 5, 5, 2),      # no overlap, dropped tail
    (200, 64, 600, 7, 7, 1),       # general hop
    (256, 256, 1100, 13, 17, 3),   # no overlap, several probes per tile (whole-series variant)
    (1024, 1024, 3100, 4, 9, 2),
    (128, 128, 1000, 6, 5, 3),
])
def test_lines_model_multi_probe(tacaw, L, H, NT, ny, nx, P):
    spec = T.SeriesSpec(P, NT, ny, nx, dtype="c64", seed=L + H, model="lines", n_terms=8,
                        amplitude=1e-3 / np.sqrt(8))
    psi = T.generate(spec)
    masks = T.standard_masks(ny, nx, scale=min(ny, nx) / 256 * 2)
    masks[3] = np.random.default_rng(1).random((ny, nx))  # custom weights
    g = run_gpu(tacaw, psi, L, H, masks)
    o = oracle_all(psi, L, H, masks=masks)
    check(g, o, label=f"L={L} H={H} NT={NT} {ny}x{nx} P={P}")
    assert g["info"]["frames_used"] == O.frames_used(NT, L, H)


@pytest.mark.parametrize("pushes,batches", [
    ([1, 7, 100, 300, 232], None),
    ([256, 256, 128], [(0, 1), (1, 3)]),
    ([640], [(0, 1), (1, 2), (2, 3)]),
    ([63, 1, 64, 512], [(0, 2), (2, 3)]),
])
def test_push_and_probe_batching_invariance(tacaw, pushes, batches):
    # App. B: the batch shape does not influence the results
    spec = T.SeriesSpec(3, 640, 10, 13, dtype="c64", seed=5, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(10, 13, scale=0.08)
    ref = run_gpu(tacaw, psi, 128, 64, masks)
    in_flight = max(p1 - p0 for p0, p1 in (batches or [(0, 3)]))
    g = run_gpu(tacaw, psi, 128, 64, masks, pushes=pushes, probe_batches=batches,
                max_probes_in_flight=in_flight)
    assert rel(g["S"], ref["S"]) < 1e-12
    assert rel(g["Dp"], ref["Dp"]) < 1e-12
    o = oracle_all(psi, 128, 64, masks=masks)
    check(g, o, label=f"pushes {pushes}")


def test_static_wave_gives_exact_zero(tacaw):
    vals = (torch.randn(1, 1, 8, 8) + 1j * torch.randn(1, 1, 8, 8)).to(torch.complex64)
    psi = vals.expand(2, 300, 8, 8).contiguous()
    g = run_gpu(tacaw, psi, 128, 64, T.standard_masks(8, 8, scale=0.05))
    assert np.all(g["S"] == 0.0) and np.all(g["D"] == 0.0) and np.all(g["Dp"] == 0.0)


@pytest.mark.parametrize("window,param,mode", [
    ("rect", None, "global"),
    ("rect", None, "none"),
    ("hann", None, "none"),
    ("hann_width", 0.8, "global"),
    ("hann_width", 1.2, "global"),
    ("tukey", 0.3, "global"),
    ("tukey", 0.5, "none"),
])
def test_windows_and_mean_modes(tacaw, window, param, mode):
    spec = T.SeriesSpec(2, 512, 9, 11, dtype="c64", seed=3, model="uniform", n_terms=3)
    psi = T.generate(spec)
    masks = T.standard_masks(9, 11, scale=0.05)
    g = run_gpu(tacaw, psi, 256, 128, masks, window=window,
                window_param=1.0 if param is None else param, mean_mode=mode)
    o = oracle_all(psi, 256, 128, window, param, masks, mode)
    check(g, o, label=f"{window} {param} {mode}")


def test_probe_sum_reduction_and_c64_c128_agree(tacaw):
    spec = T.SeriesSpec(3, 400, 8, 8, dtype="c128", seed=8, model="lines", n_terms=6)
    psi = T.generate(spec)
    g = run_gpu(tacaw, psi, 128, 64, probe_reduce="sum")
    o = oracle_all(psi, 128, 64, probe_reduce="sum")
    check(g, o, label="sum c128")
    g64 = run_gpu(tacaw, psi.to(torch.complex64), 128, 64, probe_reduce="sum")
    assert rel(g64["S"], g["S"]) < 1e-4


def test_state_and_shape_errors(tacaw):
    psi = T.generate(T.SeriesSpec(2, 400, 4, 4, seed=2)).cuda()
    plan = tacaw.Plan(2, 4, 4, 300, 128, 64, max_probes_in_flight=1)
    with pytest.raises(tacaw.TacawError) as e:
        plan.push(psi[:, :100])  # two probes streamed at once with one ring slot
    assert e.value.kind == "STATE"
    plan.push(psi[:, :300])  # whole series: no ring needed
    plan.finalize()
    plan.close()
    plan = tacaw.Plan(2, 4, 4, 300, 128, 64)
    plan.push(psi[0:1, :50], probe0=0)
    with pytest.raises(tacaw.TacawError) as e:
        plan.push(psi[:, 50:60], probe0=0)  # probes at different cursors
    assert e.value.kind == "STATE"
    with pytest.raises(tacaw.TacawError) as e:
        plan.push(psi[0:1, 50:351], probe0=0)  # 50 + 301 frames > n_frames = 300
    assert e.value.kind == "SHAPE"
    with pytest.raises(tacaw.TacawError) as e:
        plan.finalize()  # incomplete
    assert e.value.kind == "STATE"
    with pytest.raises(tacaw.TacawError) as e:
        plan.push(psi[0:1, :10], probe0=2)
    assert e.value.kind == "SHAPE"
    plan.push(psi[0:1, 50:300], probe0=0)
    plan.push(psi[1:2, :300], probe0=1)
    plan.finalize()
    with pytest.raises(tacaw.TacawError) as e:
        plan.push(psi[0:1, :10], probe0=0)
    assert e.value.kind == "STATE"
    with pytest.raises(tacaw.TacawError) as e:
        plan.finalize()
    assert e.value.kind == "STATE"
    plan.close()
    # ring capacity: two probes streamed at once with one slot
    plan = tacaw.Plan(2, 4, 4, 300, 128, 64, max_probes_in_flight=1)
    plan.push(psi[0:1, :100], probe0=0)
    with pytest.raises(tacaw.TacawError) as e:
        plan.push(psi[1:2, :100], probe0=1)
    assert e.value.kind == "STATE"
    plan.close()
    # non-compact window needs the whole series in one push
    plan = tacaw.Plan(1, 4, 4, 300, 128, 64, window="tukey", window_param=0.5)
    with pytest.raises(tacaw.TacawError) as e:
        plan.push(psi[0:1, :100])
    assert e.value.kind == "UNSUPPORTED"
    plan.close()


def test_reset_reuses_plan(tacaw):
    spec = T.SeriesSpec(2, 300, 6, 6, seed=21, model="lines")
    psi = T.generate(spec).cuda()
    plan = tacaw.Plan(2, 6, 6, 300, 128, 64)
    plan.push(psi)
    S1 = plan.finalize().clone()
    plan.reset()
    plan.push(psi)
    S2 = plan.finalize()
    torch.cuda.synchronize()
    assert torch.equal(S1, S2)
    plan.close()


def test_generator_is_bit_identical_on_gpu():
    spec = T.config_realistic(n_probe=2, n_frames=64, ny=16, nx=16)
    a = T.generate(spec, device="cuda").cpu()
    b = T.generate(spec)
    assert torch.equal(a, b)
    spec = T.config_plain_1probe()
    assert torch.equal(T.generate(spec, frames=(0, 32), device="cuda").cpu(), T.generate(spec, frames=(0, 32)))


@pytest.mark.parametrize("name,param", [
    ("blackmanharris", None), (("kaiser", 3 * np.pi), None), (("kaiser", 5 * np.pi), None),
    (("chebwin", 100), None),
])
def test_custom_windows_from_appendix(tacaw, name, param):
    # App. A compares Kaiser (beta 3 pi, 5 pi), Dolph-Chebyshev (100 dB) and
    # Blackman-Harris windows; the library takes any window as an array
    import scipy.signal

    L, H = 256, 128
    w = scipy.signal.get_window(name, L)  # periodic (DFT-even) form
    spec = T.SeriesSpec(2, 640, 8, 10, dtype="c64", seed=17, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(8, 10, scale=0.06)
    g = run_gpu(tacaw, psi, L, H, masks, window=w)
    S, Sp = O.tacaw_spectra(psi.numpy(), L, H, w)
    o = {"S": S, "D": O.detector_spectra(S, masks),
         "Dp": np.transpose(O.detector_spectra(Sp, masks), (1, 0, 2))}
    check(g, o, label=f"window {name}")


@pytest.mark.parametrize("T_K", [300.0, 50.0])
def test_quantum_statistics_factor(tacaw, T_K):
    # Eq. 1: I(q, E) ~ beta E / (1 - exp(-beta E)) |phi(q, E)|^2
    L, H, dt = 256, 128, 5.0
    spec = T.SeriesSpec(2, 512, 8, 8, dtype="c64", seed=23, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(8, 8, scale=0.05)
    g = run_gpu(tacaw, psi, L, H, masks, temperature_K=T_K, dt_fs=dt)
    q = O.quantum_factor(O.energy_axis_mev(L, dt), T_K)
    S, Sp = O.tacaw_spectra(psi.numpy(), L, H, O.window("hann", L))
    S = S * q[:, None]
    Sp = Sp * q[None, :, None]
    o = {"S": S, "D": O.detector_spectra(S, masks),
         "Dp": np.transpose(O.detector_spectra(Sp, masks), (1, 0, 2))}
    check(g, o, label=f"quantum factor T={T_K}")


def test_seg_len_200_streamed_through_the_ring(tacaw):
    # L = 200 pieces that straddle chunk boundaries: ring slots indexed by frame mod 200
    spec = T.SeriesSpec(3, 900, 8, 9, dtype="c64", seed=200, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(8, 9, scale=0.06)
    ref = run_gpu(tacaw, psi, 200, 100, masks)
    g = run_gpu(tacaw, psi, 200, 100, masks, pushes=[37, 163, 250, 1, 449],
                probe_batches=[(0, 2), (2, 3)], max_probes_in_flight=2)
    assert rel(g["S"], ref["S"]) < 1e-12 and rel(g["Dp"], ref["Dp"]) < 1e-12
    check(g, oracle_all(psi, 200, 100, masks=masks), label="L=200 streamed")
    assert g["info"]["n_segments"] == O.segment_count(900, 200, 100)


def test_seg_len_200_rejects_gemm(tacaw):
    # L = 200 has the FFT form (forward and adjoint, the adjoint tested against the
    # oracle elsewhere); the DFT-GEMM form takes powers of two only
    for tr in ("gemm_bf16x3", "gemm_f16x3"):
        with pytest.raises(tacaw.TacawError) as e:
            tacaw.Plan(1, 4, 4, 400, 200, 100, transform=tr)
        assert e.value.kind == "UNSUPPORTED"
    psi = torch.ones((1, 400, 4, 4), dtype=torch.complex64, device="cuda")
    plan = tacaw.Plan(1, 4, 4, 400, 200, 100)
    plan.push(psi)
    plan.finalize()
    g, _ = plan.backward(psi, gS=torch.zeros((200, 4, 4), dtype=torch.float64, device="cuda"))
    assert torch.count_nonzero(g).item() == 0
    plan.close()


@pytest.mark.parametrize("window", ["hann", "blackmanharris"])
def test_leakage_tails_pointwise(tacaw, window):
    # App. A compares windows by their leakage; the FP32 path must reproduce the
    # tails bin by bin, not only in the L2 norm: tones half-way between bins on an
    # elastic background, bins 4.5 .. 32.5 away from each tone
    import scipy.signal

    L, ny, nx = 512, 4, 8
    t = np.arange(L)
    nu = 40.5 + 13.0 * np.arange(ny * nx)  # one tone per pixel, all off-bin
    x = 1.0 + 1e-3 * np.exp(2j * np.pi * np.outer(t, nu) / L)
    psi = torch.from_numpy(x.astype(np.complex64).reshape(1, L, ny, nx))
    w = O.window("hann", L) if window == "hann" else scipy.signal.get_window(window, L)
    g = run_gpu(tacaw, psi, L, L, window=window if window == "hann" else w)
    So, _ = O.tacaw_spectra(psi.numpy(), L, L, w)
    # Hann tails have no zeros at half-integer offsets: compare bin by bin. The
    # Blackman-Harris transform passes near zero between its -92 dB sidelobes, so
    # there the error is measured against the tone's peak (dB below the peak).
    worst = 0.0
    for k in range(ny * nx):
        peak = So[:, k].max()
        for d in np.arange(4.5, 33.0, 1.0):
            m = int(nu[k] + d) % L
            err = abs(g["S"][m, k] - So[m, k])
            worst = max(worst, err / So[m, k] if window == "hann" else err / peak)
    say(f"{window} tails: worst {'pointwise rel' if window == 'hann' else 'rel to peak'} err {worst:.2e}")
    assert worst <= (1e-2 if window == "hann" else 1e-10)


@pytest.mark.parametrize("L,H,NT,D,pushes", [
    (128, 64, 640, 192, [64, 1, 63, 64, 64, 40, 24, 64, 64, 64, 64, 64]),  # D = L + 64: every push forces
    (128, 64, 640, 512, [100, 200, 300, 40]),                               # batches of chunks
    (128, 64, 640, 704, [512, 128]),                                         # whole series deferred
    (200, 100, 900, 300, [100] * 9),                                         # L = 200
    (256, 100, 900, 384, [128] * 7 + [4]),                                   # hop != L/2: general path
])
def test_deferred_ring_mode_matches_immediate_and_oracle(tacaw, L, H, NT, D, pushes):
    spec = T.SeriesSpec(3, NT, 9, 7, dtype="c64", seed=D + L, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(9, 7, scale=0.06)
    masks[3] = np.random.default_rng(12).random((9, 7))
    ref = run_gpu(tacaw, psi, L, H, masks)
    g = run_gpu(tacaw, psi, L, H, masks, pushes=pushes, probe_batches=[(0, 2), (2, 3)],
                max_probes_in_flight=2, ring_frames=D)
    assert rel(g["S"], ref["S"]) < 1e-12 and rel(g["Dp"], ref["Dp"]) < 1e-12
    check(g, oracle_all(psi, L, H, masks=masks), label=f"deferred L={L} H={H} D={D}")


@pytest.mark.parametrize("L,H,NT,D,ny,nx,dtype,pushes", [
    (128, 64, 640, 192, 9, 7, "c64", [64, 1, 63, 64, 64, 40, 24, 64, 64, 64, 64, 64]),
    (1024, 512, 2560, 2048, 5, 11, "c64", [512] * 5),     # 8-pixel tiles, last one padded
    (200, 100, 900, 300, 6, 9, "c64", [100] * 9),         # 32-pixel tiles
    (256, 128, 896, 512, 3, 13, "c128", [128] * 7),       # one complex128 element per store lane
])
def test_tiled_ring_matches_per_frame_ring_and_oracle(tacaw, L, H, NT, D, ny, nx, dtype, pushes):
    # the ring stored per pixel tile ([slot][tile][row][W]) gives the per-frame
    # ring's results bit for bit (same chunk arithmetic, other addresses)
    spec = T.SeriesSpec(3, NT, ny, nx, dtype=dtype, seed=D + L + 7, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(ny, nx, scale=0.06)
    masks[3] = np.random.default_rng(13).random((ny, nx))
    kw = dict(pushes=pushes, probe_batches=[(0, 2), (2, 3)], max_probes_in_flight=2,
              ring_frames=D)
    ref = run_gpu(tacaw, psi, L, H, masks, **kw)
    g = run_gpu(tacaw, psi, L, H, masks, tiled_ring=True, **kw)
    assert np.array_equal(g["S"], ref["S"]) and np.array_equal(g["Dp"], ref["Dp"])
    check(g, oracle_all(psi, L, H, masks=masks), label=f"tiled ring L={L} D={D} {dtype}")


def test_tiled_ring_rejects_ingest(tacaw):
    plan = tacaw.Plan(1, 4, 4, 640, 128, 64, ring_frames=256, tiled_ring=True)
    with pytest.raises(tacaw.TacawError) as e:
        plan.ingest(64)
    assert e.value.kind == "STATE"
    plan.close()


def test_deferred_ring_mode_errors(tacaw):
    psi = torch.ones((1, 640, 4, 4), dtype=torch.complex64, device="cuda")
    plan = tacaw.Plan(1, 4, 4, 640, 128, 64, ring_frames=256)
    with pytest.raises(tacaw.TacawError) as e:
        plan.push(psi[:, :129])  # more than ring_frames - seg_len
    assert e.value.kind == "SHAPE"
    plan.push(psi[:, :128])
    plan.close()
    with pytest.raises(tacaw.TacawError) as e:  # non-compact window: exact-mean pre-pass
        tacaw.Plan(1, 4, 4, 640, 128, 64, window="tukey", window_param=0.5, ring_frames=256)
    assert e.value.kind == "UNSUPPORTED"


@pytest.mark.parametrize("ring,tiled", [(0, False), (256, False), (256, True)])
def test_k_space_window_read_in_place(tacaw, ring, tiled):
    # Sec. II.B crops reciprocal space to a region of interest: a ny x nx window of a
    # wider grid is read in place (pixel rows k_row_stride apart), equal to the
    # reduction of the cropped copy
    big = T.generate(T.SeriesSpec(2, 640, 20, 33, dtype="c64", seed=61, model="lines", n_terms=8))
    y0, x0, ny, nx = 3, 5, 11, 17
    masks = T.standard_masks(ny, nx, scale=0.05)
    crop = big[:, :, y0:y0 + ny, x0:x0 + nx].contiguous()
    ref = run_gpu(tacaw, crop, 128, 64, masks)
    dev = big.cuda()
    view = dev[:, :, y0:y0 + ny, x0:x0 + nx]
    plan = tacaw.Plan(2, ny, nx, 640, 128, 64, masks=torch.from_numpy(masks).cuda(),
                      k_row_stride=33, ring_frames=ring, tiled_ring=tiled)
    for f0 in range(0, 640, 64):
        plan.push(view[:, f0:f0 + 64])
    S = plan.finalize().cpu().numpy().reshape(128, -1)
    D, Dp = plan.detector_spectra(per_probe=True)
    plan.close()
    assert rel(S, ref["S"]) < 1e-12 and rel(Dp.cpu().numpy(), ref["Dp"]) < 1e-12
    check({"S": S, "D": D.cpu().numpy(), "Dp": Dp.cpu().numpy()},
          oracle_all(crop, 128, 64, masks=masks), label=f"k window ring={ring} tiled={tiled}")


def test_k_space_window_adjoint(tacaw):
    from paper_2607_02236_amd import tacaw as tw

    big = T.generate(T.SeriesSpec(1, 256, 12, 20, dtype="c64", seed=62, model="lines", n_terms=8))
    y0, x0, ny, nx = 2, 3, 8, 9
    dev = big.cuda()
    view = dev[:, :, y0:y0 + ny, x0:x0 + nx]
    gS = torch.rand((128, ny, nx), dtype=torch.float64, device="cuda")
    outs = []
    for frames, rs in ((view, 20), (view.contiguous(), 0)):
        plan = tw.Plan(1, ny, nx, 256, 128, 128, k_row_stride=rs)
        plan.push(frames)
        plan.finalize()
        g, _ = plan.backward(frames, gS=gS)
        outs.append(g[:, :, :, :].contiguous().cpu().numpy())
        plan.close()
    assert np.array_equal(outs[0], outs[1])


def test_chunks_spanning_more_than_2_gib(tacaw):
    # frames 32 MiB apart (a small image inside a large frame stride): a chunk of 128
    # frames spans 4 GiB, which takes the per-row-group descriptor variant; results
    # equal the contiguous layout
    spec = T.SeriesSpec(2, 640, 8, 8, dtype="c64", seed=88, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(8, 8, scale=0.05)
    ref = run_gpu(tacaw, psi, 128, 64, masks)
    fs = (1 << 22) + 64  # elements per frame
    big = torch.empty((2, 640, fs), dtype=torch.complex64, device="cuda")
    view = big[:, :, :64].view(2, 640, 8, 8)
    view.copy_(psi.cuda())
    plan = tacaw.Plan(2, 8, 8, 640, 128, 64, masks=torch.from_numpy(masks).cuda())
    plan.push(view)
    S = plan.finalize().cpu().numpy().reshape(128, -1)
    _, Dp = plan.detector_spectra(per_probe=True)
    plan.close()
    del big
    assert rel(S, ref["S"]) < 1e-12 and rel(Dp.cpu().numpy(), ref["Dp"]) < 1e-12
