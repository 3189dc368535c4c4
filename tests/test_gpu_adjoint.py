"""GPU adjoint (hand-written backward) against the FP64 oracle's gradient and
central finite differences."""

import numpy as np
import pytest
import torch

import oracle as O
import tacaw_synth as T

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def ag():
    from paper_2607_02236_amd import autograd

    assert torch.cuda.is_available()
    return autograd


# The mean term of the gradient comes from the forward pass's bin sums when the
# window's DFT lives on bins {0, +-1} (Hann, width-r Hann at r = 1) or bin 0
# (rect), and from a separate pass otherwise (r != 1); "none" has no mean term.
@pytest.mark.parametrize("L,H,NT,ny,nx,P,mode,window,r,dtype", [
    (512, 512, 1024, 16, 16, 3, "global", "hann_width", 1.0, "c64"),  # 2 chunks of 512, no overlap
    (256, 128, 600, 9, 13, 2, "global", "hann", 1.0, "c64"),          # 50 % overlap carry, ragged
    (128, 128, 300, 8, 8, 2, "none", "hann_width", 0.8, "c64"),
    (64, 32, 200, 5, 7, 2, "global", "hann_width", 1.1, "c64"),       # mean term in a second pass
    (256, 256, 700, 6, 10, 2, "global", "rect", 1.0, "c64"),          # window DFT on bin 0 only
    (128, 64, 400, 7, 9, 2, "global", "hann", 1.0, "c128"),
    (256, 128, 700, 6, 10, 2, "global", "tukey", 0.1, "c64"),         # Sec. III.A's Tukey(0.1)
    (256, 256, 768, 6, 10, 2, "none", "tukey", 0.5, "c64"),
    (256, 128, 700, 6, 10, 2, "global", "blackmanharris", 1.0, "c64"),  # App. A, custom window
    (512, 256, 1280, 4, 8, 2, "global", "kaiser5pi", 1.0, "c64"),     # App. A, custom window
    (200, 100, 1000, 6, 10, 2, "global", "hann", 1.0, "c64"),         # the paper's L = 200 (10 x 20)
    (200, 100, 1000, 6, 10, 2, "global", "hann_width", 1.0, "c64"),
    (200, 200, 800, 5, 7, 2, "global", "hann_width", 1.1, "c64"),     # mean term in a second pass
    (200, 100, 900, 5, 7, 2, "per_segment", "hann", 1.0, "c64"),
    (200, 100, 700, 4, 9, 2, "global", "hann", 1.0, "c128"),
])
def test_adjoint_matches_oracle(ag, L, H, NT, ny, nx, P, mode, window, r, dtype):
    spec = T.SeriesSpec(P, NT, ny, nx, dtype=dtype, seed=40 + L, model="lines", n_terms=8)
    psi = T.generate(spec)
    masks = T.standard_masks(ny, nx, scale=min(ny, nx) / 128)
    masks[3] = np.random.default_rng(2).random((ny, nx))
    a = T.loss_weights(4, L, seed=4)
    b = np.random.default_rng(5).random((4, P, L)) * 0.3
    gS = np.random.default_rng(6).random((L, ny * nx)) * 0.1
    x = psi.cuda().requires_grad_(True)
    wp = torch.tensor(r, dtype=torch.float64, device="cuda", requires_grad=True)
    custom = window in ("blackmanharris", "kaiser5pi")
    if custom:  # App. A's windows, periodic, from scipy; passed as values
        import scipy.signal as ss

        spec_w = ("kaiser", 5 * np.pi) if window == "kaiser5pi" else window
        w_vals = ss.get_window(spec_w, L)
    S, D, Dp = ag.spectra(x, L, H, masks=torch.from_numpy(masks),
                          window=w_vals if custom else window, window_param=wp, mean_mode=mode)
    loss = (D * torch.from_numpy(a).cuda()).sum() + (Dp * torch.from_numpy(b).cuda()).sum() \
        + (S.reshape(L, -1) * torch.from_numpy(gS).cuda()).sum()
    loss.backward()
    w = w_vals if custom else O.window(window, L, r)
    dw = O.window_width_derivative(L, r) if window == "hann_width" else None
    Mf = masks.reshape(4, -1)
    gS_tot = gS + np.einsum("jm,jk->mk", a, Mf)
    gSp = np.einsum("jpm,jk->pmk", b, Mf)
    g_o, dr_o, lval = O.spectra_vjp(psi.numpy(), L, H, w, gS_tot, gSp, mode, dw=dw)
    assert float(loss) == pytest.approx(lval, rel=1e-5)
    e = rel(x.grad.cpu().numpy(), g_o)
    print(f"L={L} H={H} grad rel err {e:.2e}")
    assert e <= 1e-5
    if window == "hann_width":
        print(f"  dL/dr gpu {float(wp.grad):.6e} oracle {dr_o:.6e}")
        assert float(wp.grad) == pytest.approx(dr_o, rel=2e-5, abs=1e-9 * abs(lval))


def test_adjoint_directional_finite_differences(ag):
    # the loss is quadratic in psi: central differences along a random direction
    # are exact up to rounding of the FP32 forward path
    L, H, NT, ny, nx, P = 512, 512, 1024, 16, 16, 2
    spec = T.SeriesSpec(P, NT, ny, nx, dtype="c64", seed=77, model="lines", n_terms=8)
    psi = T.generate(spec).cuda()
    masks = torch.from_numpy(T.standard_masks(ny, nx, scale=ny / 128))
    a = torch.from_numpy(T.loss_weights(4, L, seed=4)).cuda()

    def loss_of(x, r=1.0):
        _, D, _ = ag.spectra(x, L, H, masks=masks, window="hann_width", window_param=r)
        return float((D * a).sum())

    x = psi.clone().requires_grad_(True)
    wp = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    _, D, _ = ag.spectra(x, L, H, masks=masks, window="hann_width", window_param=wp)
    (D * a).sum().backward()
    g = x.grad
    gen = torch.Generator(device="cpu").manual_seed(3)
    for _ in range(3):
        v = torch.complex(torch.randn(psi.shape, generator=gen), torch.randn(psi.shape, generator=gen))
        v = (v * 1e-3).to(torch.complex64).cuda()
        h = 1.0
        fd = (loss_of(psi + h * v) - loss_of(psi - h * v)) / (2 * h)
        an = float((g.conj() * v).real.sum())
        assert fd == pytest.approx(an, rel=1e-3)
    # window width: central difference with h = 1e-3 at r = 1; the support edge on
    # t = 0 makes this difference O(h) accurate (about 1e-3 relative)
    h = 1e-3
    fd = (loss_of(psi, 1 + h) - loss_of(psi, 1 - h)) / (2 * h)
    assert float(wp.grad) == pytest.approx(fd, rel=5e-3)


def test_second_backward_with_retained_graph(ag):
    # the plan stays with the graph: a second backward adds the same gradient again
    L, H, NT, ny, nx, P = 128, 64, 400, 6, 8, 2
    spec = T.SeriesSpec(P, NT, ny, nx, dtype="c64", seed=81, model="lines", n_terms=8)
    x = T.generate(spec).cuda().requires_grad_(True)
    masks = torch.from_numpy(T.standard_masks(ny, nx, scale=ny / 128))
    a = torch.from_numpy(T.loss_weights(4, L, seed=4)).cuda()
    _, D, _ = ag.spectra(x, L, H, masks=masks)
    loss = (D * a).sum()
    loss.backward(retain_graph=True)
    g1 = x.grad.clone()
    loss.backward()
    assert torch.allclose(x.grad, 2 * g1, rtol=1e-6, atol=0)
